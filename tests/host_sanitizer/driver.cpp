// Host-side setup code of libdgw under AddressSanitizer and
// UndefinedBehaviorSanitizer (test infrastructure): the reference element of
// every order, the mesh connectivity and geometry of the meshes given on the
// command line, point location, and both element orderings.  Built with g++
// from the library's host sources (no device code, no HIP calls) by
// tests/test_host_sanitizer.py.  Exit status 0 when every check passes; the
// sanitizers abort on the first error they find.
//
// usage: driver MESHFILE...   each file: int64 nvert, int64 K, int32 flags
//        (bit 0: periodic ids present), then vxyz [nvert][3] double,
//        etov [K][4] int32, pid [nvert] int32 (if flagged), face_bc [K][4] int8

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../include/dgw.h"
#include "../../paper_2205_11052_amd/csrc/dgw_internal.h"

using namespace dgw;

static int fails = 0;
#define CHECK(c, ...)                      \
  do {                                     \
    if (!(c)) {                            \
      std::fprintf(stderr, __VA_ARGS__);   \
      std::fprintf(stderr, "\n");          \
      ++fails;                             \
    }                                      \
  } while (0)

static void check_refelem() {
  for (int N = 1; N <= DGW_MAX_ORDER; ++N) {
    RefElem R;
    CHECK(build_refelem(N, R), "order %d: build_refelem failed", N);
    const int Np = (N + 1) * (N + 2) * (N + 3) / 6, Nfp = (N + 1) * (N + 2) / 2;
    CHECK(R.Np == Np && R.Nfp == Nfp, "order %d: sizes", N);
    CHECK((int)R.Dr.size() == Np * Np && (int)R.LIFT.size() == Np * 4 * Nfp,
          "order %d: operator sizes", N);
    // the basis is a partition of unity at any point, and the derivative
    // matrices annihilate constants
    const double pts[3][3] = {{-0.3, -0.2, -0.4}, {-1, -1, -1}, {0.1, -0.6, -0.5}};
    std::vector<double> l(Np);
    for (const auto &p : pts) {
      eval_basis(R, p, l.data());
      double s = 0;
      for (double v : l) s += v;
      CHECK(std::fabs(s - 1) < 1e-11, "order %d: basis sum %.17g", N, s);
    }
    for (int i = 0; i < Np; ++i) {
      double s = 0;
      for (int j = 0; j < Np; ++j) s += R.Dr[i * Np + j] + R.Ds[i * Np + j] + R.Dt[i * Np + j];
      CHECK(std::fabs(s) < 1e-9, "order %d: row %d of D not zero-sum", N, i);
    }
  }
}

static bool read_mesh(const char *path, int64_t &nvert, int64_t &K, std::vector<double> &vxyz,
                      std::vector<int32_t> &etov, std::vector<int32_t> &pid,
                      std::vector<int8_t> &bc) {
  FILE *f = std::fopen(path, "rb");
  if (!f) return false;
  int32_t flags = 0;
  bool ok = std::fread(&nvert, 8, 1, f) == 1 && std::fread(&K, 8, 1, f) == 1 &&
            std::fread(&flags, 4, 1, f) == 1;
  if (ok) {
    vxyz.resize(3 * nvert);
    etov.resize(4 * K);
    bc.resize(4 * K);
    ok = std::fread(vxyz.data(), 8, vxyz.size(), f) == vxyz.size() &&
         std::fread(etov.data(), 4, etov.size(), f) == etov.size();
    if (ok && (flags & 1)) {
      pid.resize(nvert);
      ok = std::fread(pid.data(), 4, pid.size(), f) == pid.size();
    }
    ok = ok && std::fread(bc.data(), 1, bc.size(), f) == bc.size();
  }
  std::fclose(f);
  return ok;
}

static void check_mesh(const char *path) {
  int64_t nvert = 0, K = 0;
  std::vector<double> vxyz;
  std::vector<int32_t> etov, pid;
  std::vector<int8_t> bc;
  CHECK(read_mesh(path, nvert, K, vxyz, etov, pid, bc), "%s: unreadable", path);
  if (fails) return;
  for (int N : {1, 3, 6}) {
    RefElem R;
    build_refelem(N, R);
    MeshData m;
    const std::string why = build_mesh(R, nvert, vxyz.data(), K, etov.data(),
                                       pid.empty() ? nullptr : pid.data(), bc.data(), m);
    CHECK(why.empty(), "%s order %d: %s", path, N, why.c_str());
    if (!why.empty()) continue;
    double vol = 0;
    for (double v : m.volume) vol += v;
    CHECK(vol > 0, "%s: total volume %g", path, vol);
    // the centroid of every element is found in that element (or a
    // neighbour sharing the point, lowest id first)
    for (int64_t k = 0; k < K; k += (K / 37 + 1)) {
      double x[3] = {0, 0, 0}, rst[3];
      for (int a = 0; a < 4; ++a)
        for (int d = 0; d < 3; ++d) x[d] += 0.25 * vxyz[3 * etov[4 * k + a] + d];
      const int64_t f = locate_point(m, x, rst);
      CHECK(f == k, "%s: centroid of %lld located in %lld", path, (long long)k, (long long)f);
    }
  }
  for (int method = 0; method < 2; ++method) {
    std::vector<int64_t> perm(K, -1);
    const int rc = dgw_order_elements(nvert, vxyz.data(), K, etov.data(),
                                      pid.empty() ? nullptr : pid.data(), method, perm.data());
    CHECK(rc == 0, "%s: ordering %d failed (%d)", path, method, rc);
    std::vector<char> seen(K, 0);
    for (int64_t p : perm) {
      CHECK(p >= 0 && p < K && !seen[p], "%s: ordering %d not a permutation", path, method);
      if (p >= 0 && p < K) seen[p] = 1;
    }
  }
}

int main(int argc, char **argv) {
  check_refelem();
  for (int i = 1; i < argc; ++i) check_mesh(argv[i]);
  if (fails) std::fprintf(stderr, "%d checks failed\n", fails);
  else std::printf("host checks passed\n");
  return fails ? 1 : 0;
}
