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

sigma > 0 (s = kappa^2 in lattice units; `--yukawa`): the symbol is s + 6 - 2 sum cos, and
the same expansion with 1/(s + |theta|^2)^k gives the functions g_k with (s - Lap) g_k =
g_(k-1), g_1 = e^(-kappa r)/(4 pi r): g_2 = e^(-kappa r)/(8 pi kappa),
g_3 = (1 + kappa r) e^(-kappa r)/(32 pi kappa^3).  Relative to g_1, and with u = kappa r,
x = e2/r^4, y = e3/r^6, the corrections are (fitted exactly in these invariants)
  T2 r^2 = (1 + u)(1 - 5x)/4 - u^2 x/2 + u^3 (1 - 2x)/24,
  T3 r^4 = (1 + u)(23 - 336x + 1155x^2 - 1134y)/32 + u^2 (9 - 146x + 525x^2 - 504y)/32 + ...
which at u = 0 are the q = 2 and q = 3 terms above.  The FP32 sum uses g_1 (1 + T2).
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


def yukawa():
    import random
    import mpmath as mp
    mp.mp.dps = 50
    x, y, z = sp.symbols("x y z", real=True)
    k = sp.symbols("kappa", positive=True)
    r = sp.sqrt(x * x + y * y + z * z)
    pi = sp.pi
    g1 = sp.exp(-k * r) / (4 * pi * r)
    g2 = sp.exp(-k * r) / (8 * pi * k)
    g3 = (1 + k * r) * sp.exp(-k * r) / (32 * pi * k ** 3)

    def S(f, p):
        return sum(sp.diff(f, v, p) for v in (x, y, z))

    terms = {"T2 r^2": (sp.Rational(1, 12) * S(g2, 4), 2, 3, [(0, 0), (1, 0)]),
             "T3 r^4": (sp.Rational(1, 360) * S(g2, 6) + sp.Rational(1, 144) * S(S(g3, 4), 4), 4, 6,
                        [(0, 0), (1, 0), (2, 0), (0, 1)])}
    for name, (q, rpow, udeg, kinds) in terms.items():
        f = sp.lambdify((x, y, z, k), q / g1, "mpmath")
        mons = [(d, i, j) for d in range(udeg + 1) for (i, j) in kinds]
        rows, rhs = [], []
        random.seed(7)
        for _ in range(3 * len(mons)):
            vx, vy, vz = [mp.mpf(random.uniform(-30, 30)) for _ in range(3)]
            kk = mp.mpf(random.uniform(0.001, 0.2))
            rr = mp.sqrt(vx ** 2 + vy ** 2 + vz ** 2)
            X, Y, Z = vx ** 2, vy ** 2, vz ** 2
            xh, yh = (X * Y + Y * Z + Z * X) / rr ** 4, X * Y * Z / rr ** 6
            rows.append([(kk * rr) ** d * xh ** i * yh ** j for (d, i, j) in mons])
            rhs.append(f(vx, vy, vz, kk) * rr ** rpow)
        A, b = mp.matrix(rows), mp.matrix(rhs)
        c = mp.lu_solve(A.T * A, A.T * b)
        assert mp.norm(A * c - b) / mp.norm(b) < mp.mpf(10) ** -30, "not exact in these invariants"
        print(name, "=", " + ".join(f"({sp.nsimplify(float(v), rational=True, tolerance=1e-12)})*u^{d} x^{i} y^{j}"
                                    for (d, i, j), v in zip(mons, c) if abs(v) > 1e-20))


if __name__ == "__main__":
    import sys
    yukawa() if "--yukawa" in sys.argv else main()
