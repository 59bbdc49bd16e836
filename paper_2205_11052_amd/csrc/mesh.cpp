// Host-side mesh setup: affine geometry, face matching, face node
// orientation tables and point location.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>

#include "dgw_internal.h"

namespace dgw {

namespace {

// the 6 permutations of (0, 1, 2) in lexicographic order
const int kPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2},
                         {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

void face_locals(int f, int out[3]) {
  int t = 0;
  for (int a = 0; a < 4; ++a)
    if (a != f) out[t++] = a;
}

struct FaceRec {
  std::array<int64_t, 3> key;
  int64_t k;
  int f;
};

}  // namespace

std::string build_mesh(const RefElem &R, int64_t nvert, const double *vxyz,
                       int64_t K, const int32_t *etov, const int32_t *pid,
                       const int8_t *face_bc, MeshData &m) {
  if (K <= 0 || nvert < 4) return "empty mesh";
  if (K >= (int64_t(1) << 26)) return "too many elements (limit 2^26)";
  m.K = K;
  m.vxyz.assign(vxyz, vxyz + 3 * nvert);
  m.etov.assign(etov, etov + 4 * K);
  m.geo.assign(K * DGW_META, 0.0);
  m.conn.assign(K * 4, 0);
  m.volume.assign(K, 0.0);
  m.area.assign(K * 4, 0.0);
  for (int64_t i = 0; i < 4 * K; ++i)
    if (etov[i] < 0 || etov[i] >= nvert) return "vertex id out of range";

  for (int64_t k = 0; k < K; ++k) {
    const double *v[4];
    for (int a = 0; a < 4; ++a) v[a] = vxyz + 3 * (int64_t)etov[4 * k + a];
    // X = [v1-v0, v2-v0, v3-v0] / 2 (columns)
    double X[3][3];
    for (int c = 0; c < 3; ++c)
      for (int d = 0; d < 3; ++d) X[d][c] = 0.5 * (v[c + 1][d] - v[0][d]);
    double J = X[0][0] * (X[1][1] * X[2][2] - X[1][2] * X[2][1]) -
               X[0][1] * (X[1][0] * X[2][2] - X[1][2] * X[2][0]) +
               X[0][2] * (X[1][0] * X[2][1] - X[1][1] * X[2][0]);
    if (!(J > 0) || !std::isfinite(J))
      return "element " + std::to_string(k) + " has non-positive volume";
    double *g = &m.geo[k * DGW_META];
    // inverse by cofactors: Xinv[r][b], rows are grad r, grad s, grad t
    double C[3][3];
    C[0][0] = X[1][1] * X[2][2] - X[1][2] * X[2][1];
    C[0][1] = X[0][2] * X[2][1] - X[0][1] * X[2][2];
    C[0][2] = X[0][1] * X[1][2] - X[0][2] * X[1][1];
    C[1][0] = X[1][2] * X[2][0] - X[1][0] * X[2][2];
    C[1][1] = X[0][0] * X[2][2] - X[0][2] * X[2][0];
    C[1][2] = X[0][2] * X[1][0] - X[0][0] * X[1][2];
    C[2][0] = X[1][0] * X[2][1] - X[1][1] * X[2][0];
    C[2][1] = X[0][1] * X[2][0] - X[0][0] * X[2][1];
    C[2][2] = X[0][0] * X[1][1] - X[0][1] * X[1][0];
    for (int r = 0; r < 3; ++r)
      for (int b = 0; b < 3; ++b) g[M_XINV + 3 * r + b] = C[r][b] / J;
    g[M_J] = J;
    m.volume[k] = J * 4.0 / 3.0;
    for (int f = 0; f < 4; ++f) {
      int fl[3];
      face_locals(f, fl);
      double e1[3], e2[3], cr[3], to_opp[3];
      for (int d = 0; d < 3; ++d) {
        e1[d] = v[fl[1]][d] - v[fl[0]][d];
        e2[d] = v[fl[2]][d] - v[fl[0]][d];
        to_opp[d] = v[f][d] - v[fl[0]][d];
      }
      cr[0] = e1[1] * e2[2] - e1[2] * e2[1];
      cr[1] = e1[2] * e2[0] - e1[0] * e2[2];
      cr[2] = e1[0] * e2[1] - e1[1] * e2[0];
      double len = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
      double s = (cr[0] * to_opp[0] + cr[1] * to_opp[1] + cr[2] * to_opp[2]) > 0
                     ? -1.0 : 1.0;
      for (int d = 0; d < 3; ++d) g[M_NORMAL + 3 * f + d] = s * cr[d] / len;
      m.area[4 * k + f] = 0.5 * len;
      g[M_FSCALE + f] = 0.5 * len / J;
    }
  }

  // face matching on the sorted (identified) vertex triples
  auto gid = [&](int64_t k, int a) -> int64_t {
    int64_t v = etov[4 * k + a];
    return pid ? (int64_t)pid[v] : v;
  };
  std::vector<FaceRec> faces;
  faces.reserve(4 * K);
  for (int64_t k = 0; k < K; ++k)
    for (int f = 0; f < 4; ++f) {
      int fl[3];
      face_locals(f, fl);
      std::array<int64_t, 3> key = {gid(k, fl[0]), gid(k, fl[1]), gid(k, fl[2])};
      std::sort(key.begin(), key.end());
      if (key[0] == key[1] || key[1] == key[2])
        return "degenerate face (repeated identified vertex) at element " +
               std::to_string(k);
      faces.push_back({key, k, f});
    }
  std::sort(faces.begin(), faces.end(), [](const FaceRec &a, const FaceRec &b) {
    if (a.key != b.key) return a.key < b.key;
    if (a.k != b.k) return a.k < b.k;
    return a.f < b.f;
  });
  for (size_t i = 0; i < faces.size();) {
    size_t j = i + 1;
    while (j < faces.size() && faces[j].key == faces[i].key) ++j;
    if (j - i > 2) return "non-manifold face (shared by more than 2 elements)";
    if (j - i == 2) {
      for (int side = 0; side < 2; ++side) {
        const FaceRec &A = faces[i + side], &B = faces[i + 1 - side];
        int la[3], lb[3];
        face_locals(A.f, la);
        face_locals(B.f, lb);
        int pi[3];
        for (int u = 0; u < 3; ++u) {
          pi[u] = -1;
          for (int w = 0; w < 3; ++w)
            if (gid(B.k, lb[w]) == gid(A.k, la[u])) pi[u] = w;
          if (pi[u] < 0) return "face vertex mismatch";
        }
        int o = -1;
        for (int p = 0; p < 6; ++p)
          if (kPerm[p][0] == pi[0] && kPerm[p][1] == pi[1] && kPerm[p][2] == pi[2])
            o = p;
        m.conn[4 * A.k + A.f] = (int32_t)((B.k << 5) | (B.f << 3) | o);
      }
    } else {
      const FaceRec &A = faces[i];
      int bc = face_bc ? face_bc[4 * A.k + A.f] : 0;
      if (bc == 1)
        m.conn[4 * A.k + A.f] = CONN_FREE;
      else if (bc == 2)
        m.conn[4 * A.k + A.f] = CONN_ABSORB;
      else
        return "unmatched face without a boundary tag at element " +
               std::to_string(A.k);
    }
    i = j;
  }

  // neighbour node tables nbtab[f][f2][o][m]
  const int N = R.N, Np = R.Np, Nfp = R.Nfp;
  std::vector<int> lat((N + 1) * (N + 1) * (N + 1), -1);
  for (int n = 0; n < Np; ++n)
    lat[(R.bary[4 * n + 1] * (N + 1) + R.bary[4 * n + 2]) * (N + 1) +
        R.bary[4 * n + 3]] = n;
  m.nbtab.assign(4 * 4 * 6 * Nfp, -1);
  m.nbface.assign(4 * 4 * 6 * Nfp, -1);
  for (int f = 0; f < 4; ++f)
    for (int f2 = 0; f2 < 4; ++f2)
      for (int o = 0; o < 6; ++o)
        for (int mm = 0; mm < Nfp; ++mm) {
          int la[3], lb[3];
          face_locals(f, la);
          face_locals(f2, lb);
          int n = R.fmask[f * Nfp + mm];
          int B[4] = {0, 0, 0, 0};
          for (int u = 0; u < 3; ++u) B[lb[kPerm[o][u]]] = R.bary[4 * n + la[u]];
          int idx = lat[(B[1] * (N + 1) + B[2]) * (N + 1) + B[3]];
          m.nbtab[((f * 4 + f2) * 6 + o) * Nfp + mm] = idx;
          for (int q = 0; q < Nfp; ++q)
            if (R.fmask[f2 * Nfp + q] == idx)
              m.nbface[((f * 4 + f2) * 6 + o) * Nfp + mm] = q;
        }
  // the same lookups resolved per element face node: the neighbour's
  // volume node (Np <= 84 fits a byte) and its face node f2 Nfp + m2
  // (4 Nfp <= 112 fits a byte)
  m.nbnode.assign((size_t)K * 4 * Nfp, 0);
  m.nbfnode.assign((size_t)K * 4 * Nfp, 0);
  for (int64_t k = 0; k < K; ++k)
    for (int f = 0; f < 4; ++f) {
      const int32_t cn = m.conn[4 * k + f];
      if (cn < 0) continue;
      const int f2 = (cn >> 3) & 3, o = cn & 7;
      for (int mm = 0; mm < Nfp; ++mm) {
        const int tab = ((f * 4 + f2) * 6 + o) * Nfp + mm;
        m.nbnode[(size_t)(4 * k + f) * Nfp + mm] = (uint8_t)m.nbtab[tab];
        m.nbfnode[(size_t)(4 * k + f) * Nfp + mm] = (uint8_t)(f2 * Nfp + m.nbface[tab]);
      }
    }
  return "";
}

int64_t locate_point(const MeshData &m, const double x[3], double rst[3]) {
  for (int64_t k = 0; k < m.K; ++k) {
    const double *g = &m.geo[k * DGW_META];
    const double *v0 = &m.vxyz[3 * (int64_t)m.etov[4 * k]];
    double d[3] = {x[0] - v0[0], x[1] - v0[1], x[2] - v0[2]};
    double l[3];
    for (int r = 0; r < 3; ++r)
      l[r] = 0.5 * (g[M_XINV + 3 * r] * d[0] + g[M_XINV + 3 * r + 1] * d[1] +
                    g[M_XINV + 3 * r + 2] * d[2]);
    double l0 = 1.0 - l[0] - l[1] - l[2];
    const double tol = -1e-12;
    if (l[0] >= tol && l[1] >= tol && l[2] >= tol && l0 >= tol) {
      for (int r = 0; r < 3; ++r) rst[r] = 2.0 * l[r] - 1.0;
      return k;
    }
  }
  return -1;
}

}  // namespace dgw
