// Reference tetrahedron operators, computed on the host in long double.
//
// Lagrange basis on the equispaced lattice in closed form (Silvester 1969):
// for the node with integer barycentrics (a0, a1, a2, a3), sum = N,
//     l(lam) = prod_a R_{a_a}(lam_a),   R_m(z) = prod_{j<m} (N z - j) / (j+1),
// which is 1 at its own node and 0 at every other lattice node.  Gradients
// follow from the product rule and d lam_a / d(r,s,t).  Mass and face-mass
// matrices are integrated with collapsed (Duffy) Gauss-Legendre rules of
// N+2 points per direction, exact for the polynomial integrands.
// LIFT = M^-1 [E_0 .. E_3] by a Cholesky solve.
#include <cmath>
#include <vector>

#include "dgw_internal.h"

namespace dgw {

namespace {

typedef long double ld;

void gauss_legendre(int n, std::vector<ld> &x, std::vector<ld> &w) {
  // Newton iteration on P_n from the Chebyshev-like initial guesses; the
  // nodes on [-1, 1] are mapped to [0, 1] by the caller.
  x.assign(n, 0);
  w.assign(n, 0);
  const ld pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < n; ++i) {
    ld z = std::cos(pi * (i + 0.75L) / (n + 0.5L));
    ld dp = 0;
    for (int it = 0; it < 100; ++it) {
      ld p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        ld p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1; }
      dp = n * (z * p1 - p0) / (z * z - 1);
      ld dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-30L) break;
    }
    // recompute derivative at the converged root
    ld p0 = 1, p1 = z;
    for (int k = 2; k <= n; ++k) {
      ld p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1);
    x[i] = z;
    w[i] = 2 / ((1 - z * z) * dp * dp);
  }
}

struct Lattice {
  int N, Np, Nfp;
  std::vector<int> bary;   // [Np][4] integer barycentrics
  std::vector<int> fmask;  // [4][Nfp]
};

Lattice make_lattice(int N) {
  Lattice L;
  L.N = N;
  for (int k = 0; k <= N; ++k)
    for (int j = 0; j + k <= N; ++j)
      for (int i = 0; i + j + k <= N; ++i) {
        L.bary.push_back(N - i - j - k);
        L.bary.push_back(i);
        L.bary.push_back(j);
        L.bary.push_back(k);
      }
  L.Np = (int)L.bary.size() / 4;
  L.Nfp = (N + 1) * (N + 2) / 2;
  for (int f = 0; f < 4; ++f)
    for (int n = 0; n < L.Np; ++n)
      if (L.bary[4 * n + f] == 0) L.fmask.push_back(n);
  return L;
}

// R_m(z) and its derivative
void rfun(int N, int m, ld z, ld &val, ld &der) {
  val = 1;
  der = 0;
  for (int j = 0; j < m; ++j) {
    ld fac = (N * z - j) / (j + 1);
    der = der * fac + val * (ld)N / (j + 1);
    val *= fac;
  }
}

// value and d/d(lam_0..lam_3) (lam independent) of basis function n
void basis(const Lattice &L, int n, const ld lam[4], ld &val, ld dl[4]) {
  ld v[4], d[4];
  for (int a = 0; a < 4; ++a) rfun(L.N, L.bary[4 * n + a], lam[a], v[a], d[a]);
  val = v[0] * v[1] * v[2] * v[3];
  for (int a = 0; a < 4; ++a) {
    ld p = d[a];
    for (int b = 0; b < 4; ++b)
      if (b != a) p *= v[b];
    dl[a] = p;
  }
}

bool cholesky_solve(int n, std::vector<ld> A, std::vector<ld> &B, int nrhs) {
  for (int j = 0; j < n; ++j) {
    ld s = A[j * n + j];
    for (int k = 0; k < j; ++k) s -= A[j * n + k] * A[j * n + k];
    if (!(s > 0)) return false;
    A[j * n + j] = std::sqrt(s);
    for (int i = j + 1; i < n; ++i) {
      ld t = A[i * n + j];
      for (int k = 0; k < j; ++k) t -= A[i * n + k] * A[j * n + k];
      A[i * n + j] = t / A[j * n + j];
    }
  }
  for (int c = 0; c < nrhs; ++c) {
    for (int i = 0; i < n; ++i) {
      ld t = B[i * nrhs + c];
      for (int k = 0; k < i; ++k) t -= A[i * n + k] * B[k * nrhs + c];
      B[i * nrhs + c] = t / A[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      ld t = B[i * nrhs + c];
      for (int k = i + 1; k < n; ++k) t -= A[k * n + i] * B[k * nrhs + c];
      B[i * nrhs + c] = t / A[i * n + i];
    }
  }
  return true;
}

}  // namespace

bool build_refelem(int N, RefElem &R) {
  if (N < 1 || N > DGW_MAX_ORDER) return false;
  Lattice L = make_lattice(N);
  const int Np = L.Np, Nfp = L.Nfp;
  R.N = N;
  R.Np = Np;
  R.Nfp = Nfp;
  R.bary = L.bary;
  R.fmask = L.fmask;
  R.rst.resize(Np * 3);
  for (int n = 0; n < Np; ++n)
    for (int d = 0; d < 3; ++d)
      R.rst[n * 3 + d] = -1.0 + 2.0 * L.bary[4 * n + 1 + d] / (double)N;

  // differentiation matrices: d/dr = (d/dlam1 - d/dlam0) / 2, etc.
  std::vector<ld> D[3];
  for (int d = 0; d < 3; ++d) D[d].assign(Np * Np, 0);
  for (int i = 0; i < Np; ++i) {
    ld lam[4];
    for (int a = 0; a < 4; ++a) lam[a] = (ld)L.bary[4 * i + a] / N;
    for (int n = 0; n < Np; ++n) {
      ld v, dl[4];
      basis(L, n, lam, v, dl);
      for (int d = 0; d < 3; ++d) D[d][i * Np + n] = (dl[1 + d] - dl[0]) / 2;
    }
  }

  // collapsed Gauss-Legendre rule on the unit simplex
  const int nq = N + 2;
  std::vector<ld> gx, gw;
  gauss_legendre(nq, gx, gw);
  for (int i = 0; i < nq; ++i) {
    gx[i] = (gx[i] + 1) / 2;
    gw[i] = gw[i] / 2;
  }
  // mass matrix: int over reference tet = 8 * int over unit simplex
  std::vector<ld> M(Np * Np, 0), phi(Np);
  for (int a = 0; a < nq; ++a)
    for (int b = 0; b < nq; ++b)
      for (int c = 0; c < nq; ++c) {
        ld u = gx[a], v = gx[b], w = gx[c];
        ld l1 = u, l2 = v * (1 - u), l3 = w * (1 - u) * (1 - v);
        ld wt = gw[a] * gw[b] * gw[c] * (1 - u) * (1 - u) * (1 - v) * 8;
        ld lam[4] = {1 - l1 - l2 - l3, l1, l2, l3};
        for (int n = 0; n < Np; ++n) {
          ld dl[4];
          basis(L, n, lam, phi[n], dl);
        }
        for (int i = 0; i < Np; ++i)
          for (int j = 0; j < Np; ++j) M[i * Np + j] += wt * phi[i] * phi[j];
      }

  // area-normalised face mass: (1/|F|) int_F l_i l_j = 2 * int over the unit
  // triangle in the face's own barycentrics
  std::vector<ld> E(Np * 4 * Nfp, 0);
  for (int f = 0; f < 4; ++f) {
    int fv[3], t = 0;
    for (int a = 0; a < 4; ++a)
      if (a != f) fv[t++] = a;
    for (int a = 0; a < nq; ++a)
      for (int b = 0; b < nq; ++b) {
        ld u = gx[a], v = gx[b];
        ld m1 = u, m2 = v * (1 - u), m0 = 1 - m1 - m2;
        ld wt = gw[a] * gw[b] * (1 - u) * 2;
        ld lam[4] = {0, 0, 0, 0};
        lam[fv[0]] = m0;
        lam[fv[1]] = m1;
        lam[fv[2]] = m2;
        for (int n = 0; n < Np; ++n) {
          ld dl[4];
          basis(L, n, lam, phi[n], dl);
        }
        for (int i = 0; i < Np; ++i)
          for (int m = 0; m < Nfp; ++m)
            E[i * 4 * Nfp + f * Nfp + m] += wt * phi[i] * phi[L.fmask[f * Nfp + m]];
      }
  }
  std::vector<ld> LIFT = E;
  if (!cholesky_solve(Np, M, LIFT, 4 * Nfp)) return false;

  R.Dr.resize(Np * Np);
  R.Ds.resize(Np * Np);
  R.Dt.resize(Np * Np);
  R.M.resize(Np * Np);
  R.LIFT.resize(Np * 4 * Nfp);
  for (int i = 0; i < Np * Np; ++i) {
    R.Dr[i] = (double)D[0][i];
    R.Ds[i] = (double)D[1][i];
    R.Dt[i] = (double)D[2][i];
    R.M[i] = (double)M[i];
  }
  for (int i = 0; i < Np * 4 * Nfp; ++i) R.LIFT[i] = (double)LIFT[i];
  // M^-1 for the source projection
  std::vector<ld> Minv(Np * Np, 0);
  for (int i = 0; i < Np; ++i) Minv[i * Np + i] = 1;
  if (!cholesky_solve(Np, M, Minv, Np)) return false;
  R.Minv.resize(Np * Np);
  for (int i = 0; i < Np * Np; ++i) R.Minv[i] = (double)Minv[i];
  return true;
}

void eval_basis(const RefElem &R, const double rst[3], double *out) {
  Lattice L;
  L.N = R.N;
  L.bary = R.bary;
  ld lam[4] = {0, ((ld)rst[0] + 1) / 2, ((ld)rst[1] + 1) / 2,
               ((ld)rst[2] + 1) / 2};
  lam[0] = 1 - lam[1] - lam[2] - lam[3];
  for (int n = 0; n < R.Np; ++n) {
    ld v, dl[4];
    basis(L, n, lam, v, dl);
    out[n] = (double)v;
  }
}

}  // namespace dgw
