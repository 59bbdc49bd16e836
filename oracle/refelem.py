"""Reference tetrahedron and nodal operators in exact rational arithmetic.

Oracle (test infrastructure).  The paper (arXiv 2205.11052) does not describe
the DG discretisation; everything here is the textbook nodal DG construction
(Hesthaven and Warburton, Nodal Discontinuous Galerkin Methods, 2008) written
out in exact arithmetic so that no floating-point step precedes the final
rounding to FP64.

Reference tetrahedron: vertices v0 = (-1,-1,-1), v1 = (1,-1,-1),
v2 = (-1,1,-1), v3 = (-1,-1,1), volume 4/3.  Barycentric coordinates
l1 = (1+r)/2, l2 = (1+s)/2, l3 = (1+t)/2, l0 = 1 - l1 - l2 - l3.  Face f is
the face opposite vertex f (where l_f = 0).

Nodes: the equispaced lattice of order N, node (i, j, k), i + j + k <= N, at
barycentrics (l1, l2, l3) = (i, j, k)/N, ordered k outermost, then j, then i.
Face f's nodes are the lattice nodes with l_f = 0, in ascending node order.

Polynomial basis used for the exact construction: monomials
l1^a l2^b l3^c with a + b + c <= N (they span P_N).  Exact integrals:

* volume:  int_T l0^a0 l1^a1 l2^a2 l3^a3 dV = 3! |T| a0!a1!a2!a3! / (3+sum a)!
* face:    int_F m0^b0 m1^b1 m2^b2 dA / |F| = 2! b0!b1!b2! / (2+sum b)!
  for the face's own barycentrics m0, m1, m2.

Operators (i = row node, n = column node, l_n the Lagrange basis):

* Dr[i, n] = d l_n / dr at node i, likewise Ds, Dt;
* M[i, n] = int_T l_i l_n dV (reference mass matrix);
* E_f[i, m] = (1/|F_f|) int_{F_f} l_i l_{Fmask_f[m]} dA  (area-normalised
  face mass, so every entry is rational, also on the slanted face 0);
* LIFT = M^{-1} [E_0 E_1 E_2 E_3]  (Np x 4 Nfp).

With these, the face term of the strong form on a physical element of
Jacobian J (= volume / (4/3)) and face areas A_f is
(A_f / J) * LIFT_f @ (flux at the face nodes).
"""

from fractions import Fraction
from functools import lru_cache
from math import factorial, gcd

import numpy as np

VREF = Fraction(4, 3)


def lattice(N):
    """Lattice triples (i, j, k) in node order."""
    out = []
    for k in range(N + 1):
        for j in range(N + 1 - k):
            for i in range(N + 1 - j - k):
                out.append((i, j, k))
    return out


def np_nfp(N):
    return (N + 1) * (N + 2) * (N + 3) // 6, (N + 1) * (N + 2) // 2


def lattice_barycentric(N):
    """Integer barycentrics (b0, b1, b2, b3), summing to N, per node."""
    return [(N - i - j - k, i, j, k) for (i, j, k) in lattice(N)]


def face_masks(N):
    """Fmask[f] = list of node indices on face f (l_f = 0), ascending."""
    bary = lattice_barycentric(N)
    return [[n for n, b in enumerate(bary) if b[f] == 0] for f in range(4)]


def _inverse(A):
    """Exact inverse of a square matrix of Fractions (Gauss-Jordan)."""
    n = len(A)
    M = [list(row) + [Fraction(int(i == j)) for j in range(n)]
         for i, row in enumerate(A)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        pv = M[c][c]
        M[c] = [x / pv for x in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                fct = M[r][c]
                M[r] = [x - fct * y for x, y in zip(M[r], M[c])]
    return [row[n:] for row in M]


def _transpose(A):
    return [list(r) for r in zip(*A)]


def _common(A):
    """Write a Fraction matrix as (integer matrix, common denominator)."""
    den = 1
    for row in A:
        for x in row:
            den = den * x.denominator // gcd(den, x.denominator)
    return [[x.numerator * (den // x.denominator) for x in row]
            for row in A], den


def _imatmul(A, B):
    Bt = list(zip(*B))
    return [[sum(a * b for a, b in zip(row, col)) for col in Bt] for row in A]


def _prod(A, B):
    """Exact A @ B for Fraction matrices, through integer products."""
    ia, da = _common(A)
    ib, db = _common(B)
    den = da * db
    return [[Fraction(x, den) for x in row] for row in _imatmul(ia, ib)]


def _triple(At, G, B):
    """Exact At @ G @ B for Fraction matrices, through integer products."""
    ia, da = _common(At)
    ig, dg = _common(G)
    ib, db = _common(B)
    P = _imatmul(ia, _imatmul(ig, ib))
    den = da * dg * db
    return [[Fraction(x, den) for x in row] for row in P]


def _vol_integral(a):
    """int_T l1^a1 l2^a2 l3^a3 dV over the reference tetrahedron."""
    a1, a2, a3 = a
    return (6 * VREF * factorial(a1) * factorial(a2) * factorial(a3)
            / factorial(3 + a1 + a2 + a3))


def _face_integral(f, a):
    """(1/|F_f|) int_{F_f} l1^a1 l2^a2 l3^a3 dA.

    On face f >= 1 the monomial vanishes unless a_f = 0; the remaining two
    exponents belong to two of the face's own barycentrics (the third, l0, has
    exponent 0).  On face 0 the face barycentrics are exactly (l1, l2, l3)."""
    a = list(a)
    if f >= 1:
        if a[f - 1] != 0:
            return Fraction(0)
        b = [x for i, x in enumerate(a) if i != f - 1] + [0]
    else:
        b = a
    return Fraction(2 * factorial(b[0]) * factorial(b[1]) * factorial(b[2]),
                    factorial(2 + sum(b)))


@lru_cache(maxsize=None)
def exact_operators(N):
    """Exact rational operators for order N (cached).

    Returns a dict of nested lists of Fractions: Dr, Ds, Dt, M, Minv, E
    (Np x 4Nfp, faces concatenated), LIFT, Vinv (monomial coefficients of
    the Lagrange basis, [monomial][node]), and the integer data lattice,
    Fmask, exps (monomial exponents)."""
    if N < 1:
        raise ValueError("order must be >= 1")
    P = lattice(N)
    exps = lattice(N)            # exponents (a1, a2, a3) with sum <= N
    Np = len(P)
    lam = [(Fraction(i, N), Fraction(j, N), Fraction(k, N)) for i, j, k in P]

    def mono(e, x):
        return x[0] ** e[0] * x[1] ** e[1] * x[2] ** e[2]

    def dmono(e, x, d):
        # d/dr = (1/2) d/dl1 etc.
        if e[d] == 0:
            return Fraction(0)
        ee = list(e)
        ee[d] -= 1
        return Fraction(e[d], 2) * mono(ee, x)

    V = [[mono(e, x) for e in exps] for x in lam]
    Vinv = _inverse(V)                                      # [mono][node]
    D = []
    for d in range(3):
        Vd = [[dmono(e, x, d) for e in exps] for x in lam]
        D.append(_prod(Vd, Vinv))
    G = [[_vol_integral(tuple(a + b for a, b in zip(ea, eb))) for eb in exps]
         for ea in exps]
    VinvT = _transpose(Vinv)
    M = _triple(VinvT, G, Vinv)
    Minv = _inverse(M)
    Fmask = face_masks(N)
    Ecols = []
    for f in range(4):
        Gf = [[_face_integral(f, tuple(a + b for a, b in zip(ea, eb)))
               for eb in exps] for ea in exps]
        Vf = [[Vinv[b][m] for m in Fmask[f]] for b in range(Np)]
        Ef = _triple(VinvT, Gf, Vf)                         # [node][face node]
        for c in range(len(Fmask[f])):
            Ecols.append([Ef[i][c] for i in range(Np)])
    E = _transpose(Ecols)                                   # Np x 4Nfp
    LIFT = _prod(Minv, E)
    return dict(Dr=D[0], Ds=D[1], Dt=D[2], M=M, Minv=Minv, E=E, LIFT=LIFT,
                Vinv=Vinv, lattice=P, Fmask=Fmask, exps=exps, N=N)


def to_float(A):
    return np.array([[float(x) for x in row] for row in A], dtype=np.float64)


@lru_cache(maxsize=None)
def operators(N):
    """FP64 operators, each entry the exact rational rounded once."""
    ex = exact_operators(N)
    out = {k: to_float(ex[k]) for k in ("Dr", "Ds", "Dt", "M", "Minv", "E",
                                        "LIFT", "Vinv")}
    out["Fmask"] = np.array(ex["Fmask"], dtype=np.int64)    # [4, Nfp]
    out["exps"] = np.array(ex["exps"], dtype=np.int64)
    out["lattice"] = np.array(ex["lattice"], dtype=np.int64)
    out["N"] = N
    out["Np"], out["Nfp"] = np_nfp(N)
    return out


def lagrange_at(N, rst):
    """Values of the Lagrange basis at reference points rst [P, 3] -> [P, Np].

    The Lagrange basis is l_n = sum_b Vinv[b, n] * monomial_b(l1, l2, l3).
    Each FP64 input coordinate is taken as the exact binary rational it
    represents, the basis is evaluated exactly, and the result rounded once."""
    ex = exact_operators(N)
    rst = np.atleast_2d(np.asarray(rst, dtype=np.float64))
    out = np.empty((rst.shape[0], len(ex["lattice"])), dtype=np.float64)
    for p, x in enumerate(rst):
        lam = [(1 + Fraction(float(c))) / 2 for c in x]
        mono = [lam[0] ** e[0] * lam[1] ** e[1] * lam[2] ** e[2]
                for e in ex["exps"]]
        for n in range(out.shape[1]):
            out[p, n] = float(sum((mono[b] * ex["Vinv"][b][n]
                                   for b in range(len(mono))), Fraction(0)))
    return out
