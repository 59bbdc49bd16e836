// Element orderings for gather locality (host only).
//
// The stage kernel processes blocks of consecutive elements and gives each
// XCD one contiguous range of blocks, so face neighbours that are close in
// the element numbering are read from the same L2.  An arbitrary mesh
// numbering (a mesh generator's output, a partitioner's) scatters them; the
// two orderings here restore locality:
//   * Morton (Z-order) curve of the element centroids: 21 bits per axis over
//     the centroids' bounding box, bits interleaved x, y, z from the least
//     significant end; ties by input index;
//   * reverse Cuthill-McKee on the face-adjacency graph (Cuthill and McKee,
//     Proc. 24th ACM National Conference, 1969; reversed as proposed by
//     George, 1971): breadth-first from a minimum-degree element of each
//     connected component, neighbours queued by increasing degree then
//     index, and the whole sequence reversed.
#include <algorithm>
#include <array>
#include <cstdint>
#include <numeric>
#include <vector>

#include "../../include/dgw.h"

namespace {

// spread the low 21 bits of x to every third bit
uint64_t spread3(uint64_t x) {
  x &= 0x1fffffull;
  x = (x | x << 32) & 0x1f00000000ffffull;
  x = (x | x << 16) & 0x1f0000ff0000ffull;
  x = (x | x << 8) & 0x100f00f00f00f00full;
  x = (x | x << 4) & 0x10c30c30c30c30c3ull;
  x = (x | x << 2) & 0x1249249249249249ull;
  return x;
}

void morton(int64_t K, const double *vxyz, const int32_t *etov, int64_t *perm) {
  std::vector<std::array<double, 3>> c((size_t)K);
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t k = 0; k < K; ++k) {
    for (int d = 0; d < 3; ++d) {
      double s = 0;
      for (int a = 0; a < 4; ++a) s += vxyz[3 * (int64_t)etov[4 * k + a] + d];
      c[k][d] = 0.25 * s;
      lo[d] = std::min(lo[d], c[k][d]);
      hi[d] = std::max(hi[d], c[k][d]);
    }
  }
  const double top = (double)((1 << 21) - 1);
  std::vector<uint64_t> key((size_t)K);
  for (int64_t k = 0; k < K; ++k) {
    uint64_t ix[3];
    for (int d = 0; d < 3; ++d) {
      const double w = hi[d] - lo[d];
      double t = w > 0 ? (c[k][d] - lo[d]) / w * top : 0.0;
      t = std::min(std::max(t, 0.0), top);
      ix[d] = (uint64_t)t;
    }
    key[k] = spread3(ix[0]) | spread3(ix[1]) << 1 | spread3(ix[2]) << 2;
  }
  std::iota(perm, perm + K, (int64_t)0);
  std::sort(perm, perm + K, [&](int64_t a, int64_t b) {
    return key[a] != key[b] ? key[a] < key[b] : a < b;
  });
}

// Face neighbours nb[k][f] (-1 on a face no other element shares), faces
// matched by their sorted (identified) vertex triples.  Returns false for a
// degenerate face or a triple shared by more than two faces.
bool face_graph(int64_t K, const int32_t *etov, const int32_t *pid,
                std::vector<std::array<int64_t, 4>> &nb) {
  struct FaceKey {
    int64_t v[3];
    int64_t k;
    int f;
  };
  std::vector<FaceKey> fk((size_t)K * 4);
  for (int64_t k = 0; k < K; ++k)
    for (int f = 0; f < 4; ++f) {
      int64_t v[3];
      int n = 0;
      for (int a = 0; a < 4; ++a)
        if (a != f) {
          const int64_t g = etov[4 * k + a];
          v[n++] = pid ? (int64_t)pid[g] : g;
        }
      std::sort(v, v + 3);
      if (v[0] == v[1] || v[1] == v[2]) return false;
      fk[4 * k + f] = {{v[0], v[1], v[2]}, k, f};
    }
  std::sort(fk.begin(), fk.end(), [](const FaceKey &a, const FaceKey &b) {
    for (int i = 0; i < 3; ++i)
      if (a.v[i] != b.v[i]) return a.v[i] < b.v[i];
    return a.k != b.k ? a.k < b.k : a.f < b.f;
  });
  nb.assign((size_t)K, {-1, -1, -1, -1});
  auto same = [](const FaceKey &a, const FaceKey &b) {
    return a.v[0] == b.v[0] && a.v[1] == b.v[1] && a.v[2] == b.v[2];
  };
  for (size_t i = 0; i < fk.size();) {
    size_t j = i + 1;
    while (j < fk.size() && same(fk[i], fk[j])) ++j;
    if (j - i > 2) return false;
    if (j - i == 2) {
      nb[fk[i].k][fk[i].f] = fk[i + 1].k;
      nb[fk[i + 1].k][fk[i + 1].f] = fk[i].k;
    }
    i = j;
  }
  return true;
}

void rcm(int64_t K, const std::vector<std::array<int64_t, 4>> &nb, int64_t *perm) {
  std::vector<int> deg((size_t)K, 0);
  for (int64_t k = 0; k < K; ++k)
    for (int f = 0; f < 4; ++f) deg[k] += nb[k][f] >= 0;
  auto before = [&](int64_t a, int64_t b) {
    return deg[a] != deg[b] ? deg[a] < deg[b] : a < b;
  };
  std::vector<int64_t> starts((size_t)K);
  std::iota(starts.begin(), starts.end(), (int64_t)0);
  std::sort(starts.begin(), starts.end(), before);
  std::vector<char> seen((size_t)K, 0);
  std::vector<int64_t> order;
  order.reserve((size_t)K);
  for (int64_t s : starts) {
    if (seen[s]) continue;
    seen[s] = 1;
    size_t head = order.size();
    order.push_back(s);
    while (head < order.size()) {
      const int64_t k = order[head++];
      int64_t nx[4];
      int n = 0;
      for (int f = 0; f < 4; ++f) {
        const int64_t j = nb[k][f];
        if (j >= 0 && !seen[j]) {
          seen[j] = 1;
          nx[n++] = j;
        }
      }
      std::sort(nx, nx + n, before);
      for (int i = 0; i < n; ++i) order.push_back(nx[i]);
    }
  }
  for (int64_t i = 0; i < K; ++i) perm[i] = order[(size_t)(K - 1 - i)];
}

}  // namespace

extern "C" int dgw_order_elements(int64_t nvert, const double *vxyz, int64_t K,
                                  const int32_t *etov,
                                  const int32_t *vertex_periodic_id, int method,
                                  int64_t *perm) {
  if (nvert <= 0 || K <= 0 || !vxyz || !etov || !perm) return DGW_EINVAL;
  if (method != DGW_ORDER_MORTON && method != DGW_ORDER_RCM) return DGW_EINVAL;
  for (int64_t i = 0; i < 4 * K; ++i)
    if (etov[i] < 0 || etov[i] >= nvert) return DGW_EINVAL;
  try {
    if (method == DGW_ORDER_MORTON) {
      morton(K, vxyz, etov, perm);
    } else {
      std::vector<std::array<int64_t, 4>> nb;
      if (!face_graph(K, etov, vertex_periodic_id, nb)) return DGW_EMESH;
      rcm(K, nb, perm);
    }
  } catch (...) {
    return DGW_ENOMEM;
  }
  return DGW_OK;
}
