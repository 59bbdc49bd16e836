// Anisotropic elements: the per-element data of the stage kernel's
// anisotropic form (stiffness, impedance matrices of every face, compliance)
// and its C ABI entry point.
//
// Along the normal n of a face the traction t = N(n)^T sigma and the
// velocity obey rho v_t = dt/dx_n, t_t = G dv/dx_n with the Christoffel
// matrix G = N(n)^T C N(n), N(n) the 6x3 map from a vector a to the Voigt
// strain of sym(a n^T).  With Z = (rho G)^(1/2) (symmetric positive
// definite) the combinations t - Z v and t + Z v travel along +n and -n, so
// the exact Riemann states at a face with impedance matrices Z- and Z+ are
// v* = (Z- + Z+)^-1 (Z- v- + Z+ v+ + t+ - t-) and t* = t- + Z- (v* - v-).
// For isotropic C, Z = Zp n n^T + Zs (I - n n^T): the states of the exact
// isotropic Riemann solver (Wilcox et al., J. Comput. Phys. 229, 2010).
#include <cmath>
#include <cstring>
#include <string>

#include "../../include/dgw.h"
#include "dgw_ctx.h"

using namespace dgw;

namespace {

void voigt_n(const double n[3], double Nm[6][3]) {
  std::memset(Nm, 0, sizeof(double) * 18);
  Nm[0][0] = n[0];
  Nm[1][1] = n[1];
  Nm[2][2] = n[2];
  Nm[3][1] = n[2];
  Nm[3][2] = n[1];
  Nm[4][0] = n[2];
  Nm[4][2] = n[0];
  Nm[5][0] = n[1];
  Nm[5][1] = n[0];
}

void full6(const double *up, double C[6][6]) {
  int u = 0;
  for (int a = 0; a < 6; ++a)
    for (int b = a; b < 6; ++b) C[a][b] = C[b][a] = up[u++];
}

// G = N^T C N
void christoffel(const double C[6][6], const double n[3], double G[3][3]) {
  double Nm[6][3];
  voigt_n(n, Nm);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) s += Nm[a][i] * C[a][b] * Nm[b][j];
      G[i][j] = s;
    }
}

// Eigenvalues w and eigenvectors (columns of V) of a symmetric 3x3 matrix by
// cyclic Jacobi rotations (Golub and Van Loan, Matrix Computations, 8.5).
void jacobi3(const double A0[3][3], double w[3], double V[3][3]) {
  double A[3][3];
  std::memcpy(A, A0, sizeof A);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) V[i][j] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (off <= 1e-34 * dia || off == 0.0) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        if (A[p][q] == 0.0) continue;
        const double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
        const double t = (theta >= 0 ? 1.0 : -1.0) /
                         (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < 3; ++k) {   // A <- A J (columns p, q)
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {   // A <- J^T A (rows p, q)
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) {   // V <- V J
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
  }
  for (int i = 0; i < 3; ++i) w[i] = A[i][i];
}

// Z = (rho G)^(1/2); false unless rho G is positive definite.
bool impedance(const double C[6][6], double rho, const double n[3], double Z[3][3]) {
  double G[3][3], w[3], V[3][3];
  christoffel(C, n, G);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) G[i][j] *= rho;
  jacobi3(G, w, V);
  for (int i = 0; i < 3; ++i)
    if (!(w[i] > 0)) return false;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int m = 0; m < 3; ++m) s += V[i][m] * std::sqrt(w[m]) * V[j][m];
      Z[i][j] = s;
    }
  // exactly symmetric
  for (int i = 0; i < 3; ++i)
    for (int j = i + 1; j < 3; ++j) Z[i][j] = Z[j][i] = 0.5 * (Z[i][j] + Z[j][i]);
  return true;
}

bool inverse3(const double A[3][3], double B[3][3]) {
  const double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
  const double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
  const double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
  const double det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
  if (!(std::fabs(det) > 0)) return false;
  const double id = 1.0 / det;
  B[0][0] = c00 * id;
  B[1][0] = c01 * id;
  B[2][0] = c02 * id;
  B[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) * id;
  B[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) * id;
  B[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) * id;
  B[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) * id;
  B[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) * id;
  B[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) * id;
  return true;
}

// Cholesky factor L (C = L L^T); false unless C is positive definite.
bool cholesky6(const double C[6][6], double L[6][6]) {
  std::memset(L, 0, sizeof(double) * 36);
  for (int j = 0; j < 6; ++j) {
    double d = C[j][j];
    for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
    if (!(d > 0)) return false;
    L[j][j] = std::sqrt(d);
    for (int i = j + 1; i < 6; ++i) {
      double s = C[i][j];
      for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
      L[i][j] = s / L[j][j];
    }
  }
  return true;
}

// C^-1 from its Cholesky factor, column by column.
void spd_inverse6(const double L[6][6], double S[6][6]) {
  for (int col = 0; col < 6; ++col) {
    double y[6], x[6];
    for (int i = 0; i < 6; ++i) {
      double s = i == col ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
      y[i] = s / L[i][i];
    }
    for (int i = 5; i >= 0; --i) {
      double s = y[i];
      for (int k = i + 1; k < 6; ++k) s -= L[k][i] * x[k];
      x[i] = s / L[i][i];
    }
    for (int i = 0; i < 6; ++i) S[i][col] = x[i];
  }
  for (int i = 0; i < 6; ++i)
    for (int j = i + 1; j < 6; ++j) S[i][j] = S[j][i] = 0.5 * (S[i][j] + S[j][i]);
}

void put_sym3(const double Z[3][3], double *o) {
  o[0] = Z[0][0];
  o[1] = Z[1][1];
  o[2] = Z[2][2];
  o[3] = Z[1][2];
  o[4] = Z[0][2];
  o[5] = Z[0][1];
}

}  // namespace

// Largest squared wave speed of an anisotropic element over 258 directions
// (the three axes and a Fibonacci lattice of 255 points on the sphere).
double dgw_ctx::aniso_max_speed2(int64_t k) const {
  double C[6][6];
  full6(aniso_C.data() + 21 * k, C);
  double best = 0;
  const int M = 255;
  for (int i = 0; i < M + 3; ++i) {
    double n[3];
    if (i < 3) {
      n[0] = i == 0;
      n[1] = i == 1;
      n[2] = i == 2;
    } else {
      const double z = 1.0 - (2.0 * (i - 3) + 1.0) / M;
      const double r = std::sqrt(std::fmax(0.0, 1.0 - z * z));
      const double ph = (i - 3) * 2.399963229728653;   // golden angle
      n[0] = r * std::cos(ph);
      n[1] = r * std::sin(ph);
      n[2] = z;
    }
    double G[3][3], w[3], V[3][3];
    christoffel(C, n, G);
    jacobi3(G, w, V);
    for (int m = 0; m < 3; ++m) best = std::fmax(best, w[m]);
  }
  return best / rho[k];
}

// Fill and upload the [K][DGW_ANI] table from aniso_C and rho.
int dgw_ctx::aniso_table() {
  const int64_t K = mesh.K;
  std::vector<double> t((size_t)K * DGW_ANI, 0.0);
  for (int64_t k = 0; k < K; ++k) {
    double C[6][6], L[6][6], S[6][6];
    full6(aniso_C.data() + 21 * k, C);
    if (!cholesky6(C, L))
      return fail(DGW_EINVAL, "stiffness not positive definite at element " + std::to_string(k));
    spd_inverse6(L, S);
    double *o = t.data() + k * DGW_ANI;
    int u = 0;
    for (int a = 0; a < 6; ++a)
      for (int b = a; b < 6; ++b, ++u) {
        o[A_C + u] = C[a][b];
        o[A_S + u] = S[a][b];
      }
    const double *g = mesh.geo.data() + k * DGW_META;
    for (int f = 0; f < 4; ++f) {
      const double n[3] = {g[M_NORMAL + 3 * f], g[M_NORMAL + 3 * f + 1],
                           g[M_NORMAL + 3 * f + 2]};
      const int32_t cn = mesh.conn[4 * k + f];
      double Zm[3][3], Zp[3][3], Zs[3][3], W[3][3];
      if (!impedance(C, rho[k], n, Zm))
        return fail(DGW_EINVAL, "impedance not positive definite at element " +
                                    std::to_string(k));
      if (cn >= 0) {
        const int64_t nb = cn >> 5;
        double Cn[6][6];
        full6(aniso_C.data() + 21 * nb, Cn);
        if (!impedance(Cn, rho[nb], n, Zp))
          return fail(DGW_EINVAL, "impedance not positive definite at element " +
                                      std::to_string(nb));
      } else {
        std::memcpy(Zp, Zm, sizeof Zp);
      }
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Zs[i][j] = Zm[i][j] + Zp[i][j];
      if (!inverse3(Zs, W)) return fail(DGW_EINVAL, "singular impedance sum");
      for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j) W[i][j] = W[j][i] = 0.5 * (W[i][j] + W[j][i]);
      double *fo = o + A_FACE + A_FSTRIDE * f;
      put_sym3(Zm, fo + A_ZM);
      put_sym3(W, fo + A_W);
      put_sym3(Zp, fo + A_ZP);
    }
  }
  if (!d_aniso) {
    d_aniso = (double *)dalloc(sizeof(double) * t.size());
    if (!d_aniso) return fail(DGW_ENOMEM, "device allocation failed (anisotropic data)");
  }
  return upload(d_aniso, t.data(), sizeof(double) * t.size());
}

extern "C" int dgw_set_stiffness(dgw_ctx *c, const double *C) {
  if (!c) return DGW_EINVAL;
  if (!c->have_mesh || !c->have_mat)
    return c->fail(DGW_ESTATE, "set the mesh and the material first");
  c->invalidate_graph();
  c->touch();
  if (!C) {
    c->have_aniso = false;
    c->aniso_C.clear();
    return DGW_OK;
  }
  if (c->pml_n > 0)
    return c->fail(DGW_ESTATE, "the perfectly matched layer supports isotropic elements only");
  const int64_t K = c->mesh.K;
  for (int64_t i = 0; i < 21 * K; ++i)
    if (!std::isfinite(C[i]))
      return c->fail(DGW_EINVAL, "non-finite stiffness at element " + std::to_string(i / 21));
  std::vector<double> old;
  old.swap(c->aniso_C);
  c->aniso_C.assign(C, C + 21 * K);
  int rc = c->aniso_table();
  if (rc) {
    c->aniso_C.swap(old);
    if (c->have_aniso) (void)c->aniso_table();   // restore the previous table
    return rc;
  }
  c->have_aniso = true;
  // the minimal-form kernel is isotropic only: back to the default shape
  if (c->kernel == 2) {
    c->kernel = 0;
    c->block = default_block(0, c->R.N, c->precision);
    c->wpc = 0;
  }
  return DGW_OK;
}
