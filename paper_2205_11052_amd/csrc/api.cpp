// C ABI of the dgw library (declared in include/dgw.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/dgw.h"
#include "dgw_internal.h"
#include "dgw_ctx.h"

using namespace dgw;

namespace {

// Carpenter-Kennedy five-stage fourth-order 2N-storage coefficients.
const double kRkA[5] = {0.0, -567301805773.0 / 1357537059087.0,
                        -2404267990393.0 / 2016746695238.0,
                        -3550918686646.0 / 2091501179385.0,
                        -1275806237668.0 / 842570457699.0};
const double kRkB[5] = {1432997174477.0 / 9575080441755.0,
                        5161836677717.0 / 13612068292357.0,
                        1720146321549.0 / 2090206949498.0,
                        3134564353537.0 / 4481467310338.0,
                        2277821191437.0 / 14882151754819.0};
const double kRkC[5] = {0.0, 1432997174477.0 / 9575080441755.0,
                        2526269341429.0 / 6820363962896.0,
                        2006345519317.0 / 3224310063776.0,
                        2802321613138.0 / 2924317926251.0};

}  // namespace

namespace dgw {
const double *rk_a() { return kRkA; }
const double *rk_b() { return kRkB; }
const double *rk_c() { return kRkC; }
}  // namespace dgw

int dgw_ctx::fail(int code, const std::string &msg) {
  err = msg;
  return code;
}

int dgw_ctx::hipfail(hipError_t e, const char *what) {
  err = std::string(what) + ": " + hipGetErrorString(e);
  return DGW_EHIP;
}

void *dgw_ctx::dalloc(size_t bytes) {
  if (bytes == 0) bytes = 8;
  void *p = nullptr;
  if (alloc_fn) {
    p = alloc_fn(bytes, alloc_user);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (p) owned.push_back(p);
  return p;
}

void dgw_ctx::dfree(void *p) {
  if (!p) return;
  auto it = std::find(owned.begin(), owned.end(), p);
  if (it == owned.end()) return;
  owned.erase(it);
  if (alloc_fn)
    free_fn(p, alloc_user);
  else
    (void)hipFree(p);
}

int dgw_ctx::ensure_device() {
  if (device_ready) return DGW_OK;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n <= 0) return fail(DGW_EHIP, "no HIP device available");
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) == hipSuccess) device = dev;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      cus > 0)
    ncu = cus;
  if (!stream) {
    e = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hipfail(e, "hipStreamCreate");
    own_stream = true;
  }
  device_ready = true;
  return DGW_OK;
}

int dgw_ctx::upload(void *dst, const void *src, size_t bytes) {
  hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hipfail(e, "hipMemcpyAsync H2D");
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hipfail(e, "hipStreamSynchronize");
  return DGW_OK;
}

int dgw_ctx::download(void *dst, const void *src, size_t bytes) {
  hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, stream);
  if (e != hipSuccess) return hipfail(e, "hipMemcpyAsync D2H");
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hipfail(e, "hipStreamSynchronize");
  return DGW_OK;
}

size_t dgw_ctx::real_size() const { return precision == 64 ? 8 : 4; }

void dgw_ctx::invalidate_graph() {
  if (graph_ok) {
    (void)hipGraphExecDestroy(graph_exec);
    graph_ok = false;
  }
}

template <typename real>
static std::vector<real> convert(const std::vector<double> &v) {
  return std::vector<real>(v.begin(), v.end());
}

template <typename real>
static std::vector<real> transpose(const std::vector<double> &A, int rows,
                                   int cols) {
  std::vector<real> T((size_t)rows * cols);
  for (int i = 0; i < rows; ++i)
    for (int j = 0; j < cols; ++j) T[(size_t)j * rows + i] = (real)A[(size_t)i * cols + j];
  return T;
}

int dgw_ctx::upload_operators() {
  const int Np = R.Np, NF = 4 * R.Nfp;
  const size_t rs = real_size();
  d_DrT = dalloc(rs * Np * Np);
  d_DsT = dalloc(rs * Np * Np);
  d_DtT = dalloc(rs * Np * Np);
  d_LIFTT = dalloc(rs * Np * NF);
  d_fmask = (int32_t *)dalloc(sizeof(int32_t) * NF);
  d_M = (double *)dalloc(sizeof(double) * Np * Np);
  if (!d_DrT || !d_DsT || !d_DtT || !d_LIFTT || !d_fmask || !d_M)
    return fail(DGW_ENOMEM, "device allocation failed (operators)");
  int rc;
  if (precision == 64) {
    auto a = transpose<double>(R.Dr, Np, Np), b = transpose<double>(R.Ds, Np, Np),
         c = transpose<double>(R.Dt, Np, Np), l = transpose<double>(R.LIFT, Np, NF);
    if ((rc = upload(d_DrT, a.data(), rs * a.size()))) return rc;
    if ((rc = upload(d_DsT, b.data(), rs * b.size()))) return rc;
    if ((rc = upload(d_DtT, c.data(), rs * c.size()))) return rc;
    if ((rc = upload(d_LIFTT, l.data(), rs * l.size()))) return rc;
  } else {
    auto a = transpose<float>(R.Dr, Np, Np), b = transpose<float>(R.Ds, Np, Np),
         c = transpose<float>(R.Dt, Np, Np), l = transpose<float>(R.LIFT, Np, NF);
    if ((rc = upload(d_DrT, a.data(), rs * a.size()))) return rc;
    if ((rc = upload(d_DsT, b.data(), rs * b.size()))) return rc;
    if ((rc = upload(d_DtT, c.data(), rs * c.size()))) return rc;
    if ((rc = upload(d_LIFTT, l.data(), rs * l.size()))) return rc;
  }
  // operator fragments for the matrix-core stage kernel, in MFMA lane
  // order (lane l of a 16x4 tile holds row l % 16, column l / 16), zero
  // outside the operator: Avol[a][ks][mt][l] = D_a[16 mt + l % 16][4 ks +
  // l / 16] and Alift[ks][mt][l] = LIFT[16 mt + l % 16][4 ks + l / 16]
  {
    const int MT = (Np + 15) / 16, KS = (Np + 3) / 4, KL = NF / 4;
    std::vector<double> av((size_t)3 * KS * MT * 64, 0.0), al((size_t)KL * MT * 64, 0.0);
    const std::vector<double> *D[3] = {&R.Dr, &R.Ds, &R.Dt};
    for (int a = 0; a < 3; ++a)
      for (int ks = 0; ks < KS; ++ks)
        for (int mt = 0; mt < MT; ++mt)
          for (int l = 0; l < 64; ++l) {
            const int i = 16 * mt + l % 16, j = 4 * ks + l / 16;
            if (i < Np && j < Np)
              av[(((size_t)a * KS + ks) * MT + mt) * 64 + l] = (*D[a])[(size_t)i * Np + j];
          }
    for (int ks = 0; ks < KL; ++ks)
      for (int mt = 0; mt < MT; ++mt)
        for (int l = 0; l < 64; ++l) {
          const int i = 16 * mt + l % 16, m = 4 * ks + l / 16;
          if (i < Np) al[((size_t)ks * MT + mt) * 64 + l] = R.LIFT[(size_t)i * NF + m];
        }
    // per-face lift fragments of the minimal-form kernel, scaled by the
    // face's reference coefficient (2 for face 0, -2 for faces 1-3; powers
    // of two, so the scaling is exact): Alf[f][ks][mt][l] =
    // c_f LIFT[16 mt + l % 16][f Nfp + 4 ks + l / 16], zero past Nfp
    const int Nfp = R.Nfp, KF = (Nfp + 3) / 4;
    std::vector<double> af((size_t)4 * KF * MT * 64, 0.0);
    for (int f = 0; f < 4; ++f)
      for (int ks = 0; ks < KF; ++ks)
        for (int mt = 0; mt < MT; ++mt)
          for (int l = 0; l < 64; ++l) {
            const int i = 16 * mt + l % 16, m = 4 * ks + l / 16;
            if (i < Np && m < Nfp)
              af[(((size_t)f * KF + ks) * MT + mt) * 64 + l] =
                  (f == 0 ? 2.0 : -2.0) * R.LIFT[(size_t)i * NF + f * Nfp + m];
          }
    d_Avol = dalloc(rs * av.size());
    d_Alift = dalloc(rs * al.size());
    d_Alf = dalloc(rs * af.size());
    if (!d_Avol || !d_Alift || !d_Alf)
      return fail(DGW_ENOMEM, "device allocation failed (operators)");
    if (precision == 64) {
      if ((rc = upload(d_Avol, av.data(), rs * av.size()))) return rc;
      if ((rc = upload(d_Alift, al.data(), rs * al.size()))) return rc;
      if ((rc = upload(d_Alf, af.data(), rs * af.size()))) return rc;
    } else {
      std::vector<float> avf(av.begin(), av.end()), alf(al.begin(), al.end()),
          aff(af.begin(), af.end());
      if ((rc = upload(d_Avol, avf.data(), rs * avf.size()))) return rc;
      if ((rc = upload(d_Alift, alf.data(), rs * alf.size()))) return rc;
      if ((rc = upload(d_Alf, aff.data(), rs * aff.size()))) return rc;
    }
  }
  std::vector<int32_t> fm(R.fmask.begin(), R.fmask.end());
  if ((rc = upload(d_fmask, fm.data(), sizeof(int32_t) * fm.size()))) return rc;
  if ((rc = upload(d_M, R.M.data(), sizeof(double) * R.M.size()))) return rc;
  return DGW_OK;
}

int dgw_ctx::alloc_shots() {
  const size_t n = (size_t)nshots * mesh.K * 9 * R.Np;
  const size_t rs = real_size();
  d_q[0] = dalloc(rs * n);
  d_q[1] = dalloc(rs * n);
  d_res = dalloc(rs * n);
  d_step = (int64_t *)dalloc(sizeof(int64_t) * nshots);
  d_len = (int64_t *)dalloc(sizeof(int64_t) * nshots);
  d_src_elem = (int32_t *)dalloc(sizeof(int32_t) * nshots);
  d_src_vec = (double *)dalloc(sizeof(double) * nshots * R.Np);
  d_src_par = (double *)dalloc(sizeof(double) * nshots * 10);
  if (!d_q[0] || !d_q[1] || !d_res || !d_step || !d_len || !d_src_elem ||
      !d_src_vec || !d_src_par)
    return fail(DGW_ENOMEM, "device allocation failed (fields)");
  hipError_t e;
  if ((e = hipMemsetAsync(d_q[0], 0, rs * n, stream)) != hipSuccess ||
      (e = hipMemsetAsync(d_q[1], 0, rs * n, stream)) != hipSuccess ||
      (e = hipMemsetAsync(d_res, 0, rs * n, stream)) != hipSuccess)
    return hipfail(e, "hipMemsetAsync");
  h_step.assign(nshots, 0);
  h_len.assign(nshots, std::numeric_limits<int64_t>::max());
  h_src_elem.assign(nshots, -1);
  h_src_vec.assign((size_t)nshots * R.Np, 0.0);
  h_src_par.assign((size_t)nshots * 10, 0.0);
  h_nrec.assign(nshots, 0);
  h_cap_shot.assign(nshots, 0);
  loc.assign(nshots, 0);
  cur = 0;
  // receiver counts start at zero so the sampling kernel never touches the
  // (not yet allocated) receiver tables
  d_nrec = (int32_t *)dalloc(sizeof(int32_t) * nshots);
  if (!d_nrec) return fail(DGW_ENOMEM, "device allocation failed (receivers)");
  int rc;
  if ((rc = upload(d_nrec, h_nrec.data(), sizeof(int32_t) * nshots))) return rc;
  if ((rc = sync_shot_tables())) return rc;
  return DGW_OK;
}

int dgw_ctx::sync_shot_tables() {
  int rc;
  if ((rc = upload(d_step, h_step.data(), sizeof(int64_t) * nshots))) return rc;
  if ((rc = upload(d_len, h_len.data(), sizeof(int64_t) * nshots))) return rc;
  if ((rc = upload(d_src_elem, h_src_elem.data(), sizeof(int32_t) * nshots))) return rc;
  if ((rc = upload(d_src_vec, h_src_vec.data(), sizeof(double) * h_src_vec.size()))) return rc;
  if ((rc = upload(d_src_par, h_src_par.data(), sizeof(double) * h_src_par.size()))) return rc;
  return DGW_OK;
}

int dgw_ctx::ensure_receivers(int need_r, int64_t need_cap) {
  if (need_r <= rmax && need_cap <= cap && d_trace) return DGW_OK;
  const int nr = std::max(need_r, rmax);
  const int64_t nc = std::max(need_cap, cap);
  // keep the existing contents
  std::vector<int32_t> old_elem = h_rec_elem;
  std::vector<double> old_w = h_rec_w;
  std::vector<double> old_tr;
  if (d_trace && rmax > 0 && cap > 0) {
    old_tr.resize((size_t)nshots * rmax * 3 * cap);
    int rc = download(old_tr.data(), d_trace, sizeof(double) * old_tr.size());
    if (rc) return rc;
  }
  std::vector<int32_t> ne((size_t)nshots * nr, 0);
  std::vector<double> nw((size_t)nshots * nr * R.Np, 0.0);
  std::vector<double> nt((size_t)nshots * nr * 3 * nc, 0.0);
  for (int s = 0; s < nshots; ++s)
    for (int r = 0; r < rmax; ++r) {
      ne[(size_t)s * nr + r] = old_elem[(size_t)s * rmax + r];
      for (int j = 0; j < R.Np; ++j)
        nw[((size_t)s * nr + r) * R.Np + j] = old_w[((size_t)s * rmax + r) * R.Np + j];
      if (!old_tr.empty())
        for (int c = 0; c < 3; ++c)
          for (int64_t t = 0; t < cap; ++t)
            nt[(((size_t)s * nr + r) * 3 + c) * nc + t] =
                old_tr[(((size_t)s * rmax + r) * 3 + c) * cap + t];
    }
  dfree(d_rec_elem);
  dfree(d_rec_w);
  dfree(d_trace);
  d_rec_elem = (int32_t *)dalloc(sizeof(int32_t) * ne.size());
  d_rec_w = (double *)dalloc(sizeof(double) * nw.size());
  d_trace = (double *)dalloc(sizeof(double) * nt.size());
  if (!d_nrec) d_nrec = (int32_t *)dalloc(sizeof(int32_t) * nshots);
  if (!d_rec_elem || !d_rec_w || !d_trace || !d_nrec)
    return fail(DGW_ENOMEM, "device allocation failed (receivers)");
  rmax = nr;
  cap = nc;
  h_rec_elem = ne;
  h_rec_w = nw;
  int rc;
  if ((rc = upload(d_rec_elem, ne.data(), sizeof(int32_t) * ne.size()))) return rc;
  if ((rc = upload(d_rec_w, nw.data(), sizeof(double) * nw.size()))) return rc;
  if ((rc = upload(d_trace, nt.data(), sizeof(double) * nt.size()))) return rc;
  if ((rc = upload(d_nrec, h_nrec.data(), sizeof(int32_t) * nshots))) return rc;
  invalidate_graph();
  return DGW_OK;
}

int dgw_ctx::clear_traces(int shot) {
  if (!d_trace || rmax == 0) return DGW_OK;
  const size_t n = (size_t)rmax * 3 * cap;
  hipError_t e = hipMemsetAsync(d_trace + (size_t)shot * n, 0, sizeof(double) * n, stream);
  if (e != hipSuccess) return hipfail(e, "hipMemsetAsync");
  return DGW_OK;
}

int dgw_ctx::material_meta() {
  const int64_t K = mesh.K;
  std::vector<double> &g = mesh.geo;
  for (int64_t k = 0; k < K; ++k) {
    double *m = &g[k * DGW_META];
    m[M_RHOINV] = 1.0 / rho[k];
    m[M_LAM] = lam[k];
    m[M_MU] = mu[k];
    m[47] = rho[k];
    m[M_ZP] = std::sqrt(rho[k] * (lam[k] + 2.0 * mu[k]));
    m[M_ZS] = std::sqrt(rho[k] * mu[k]);
  }
  for (int64_t k = 0; k < K; ++k) {
    double *m = &g[k * DGW_META];
    for (int f = 0; f < 4; ++f) {
      const int32_t cn = mesh.conn[4 * k + f];
      double zp = m[M_ZP], zs = m[M_ZS];
      if (cn >= 0) {
        const int64_t nb = cn >> 5;
        zp = g[nb * DGW_META + M_ZP];
        zs = g[nb * DGW_META + M_ZS];
      }
      m[M_ZPNB + f] = zp;
      m[M_ZSNB + f] = zs;
      m[M_IZPS + f] = 1.0 / (m[M_ZP] + zp);
      // both sides fluid (mu = 0): no tangential coupling (the kernel's
      // tangential Riemann amplitude is multiplied by this factor)
      m[M_IZSS + f] = m[M_ZS] + zs > 0 ? 1.0 / (m[M_ZS] + zs) : 0.0;
    }
  }
  return upload(d_meta, g.data(), sizeof(double) * g.size());
}


// Enqueue one step (5 stages + receivers) starting from buffer `from`;
// returns the buffer holding the result.
int dgw_ctx::enqueue_step(int from, bool timed) {
  for (int i = 0; i < 5; ++i) {
    hipError_t e;
    if (timed && ev_pool_used + 2 <= (int)ev_pool.size()) {
      (void)hipEventRecord(ev_pool[ev_pool_used], stream);
    }
    const int ns = slots > 0 ? slots : nshots;
    if (precision == 64) {
      StageArgs<double> a;
      stage_args(this, a, d_q[from], d_q[1 - from], d_res, d_step, i);
      a.shot_map = mapped ? d_shot_map : nullptr;
      e = launch_stage(kernel, R.N, 64, block, wpc, ncu, ns, &a, stream);
    } else {
      StageArgs<float> a;
      stage_args(this, a, d_q[from], d_q[1 - from], d_res, d_step, i);
      a.shot_map = mapped ? d_shot_map : nullptr;
      e = launch_stage(kernel, R.N, 32, block, wpc, ncu, ns, &a, stream);
    }
    if (e != hipSuccess) return hipfail(e, "stage kernel launch");
    if (timed && ev_pool_used + 2 <= (int)ev_pool.size()) {
      (void)hipEventRecord(ev_pool[ev_pool_used + 1], stream);
      ev_pool_used += 2;
    }
    if (pml_n > 0) {
      const int rc = enqueue_pml(d_q[from], d_q[1 - from], i, timed);
      if (rc) return rc;
    }
    from = 1 - from;
  }
  RecArgs r;
  r.q = d_q[from];
  r.shot_stride = mesh.K * 9 * R.Np;
  r.Np = R.Np;
  r.nrec = d_nrec;
  r.rmax = rmax;
  r.rec_elem = d_rec_elem;
  r.rec_w = d_rec_w;
  r.trace = d_trace;
  r.cap = cap;
  r.shot_step = d_step;
  r.shot_len = d_len;
  hipError_t e = launch_receivers(precision, nshots, r, stream);
  if (e != hipSuccess) return hipfail(e, "receiver kernel launch");
  return DGW_OK;
}

// The layer's launch after stage `stage` (state `in` -> `out`).
int dgw_ctx::enqueue_pml(const void *in, void *out, int stage, bool timed) {
  const bool ev = timed && pml_ev_used + 2 <= (int)pml_ev.size();
  if (ev) (void)hipEventRecord(pml_ev[pml_ev_used], stream);
  auto fill = [&](auto &a) {
    using real = std::remove_pointer_t<decltype(a.q_out)>;
    a.q_in = (const real *)in;
    a.q_out = (real *)out;
    a.res = (real *)d_res;
    a.mem = (real *)d_pml_mem;
    a.mres = (real *)d_pml_mres;
    a.elem = d_pml_elem;
    a.prof = d_pml_prof;
    a.meta = d_meta;
    a.conn = d_conn;
    a.nbnode = d_nbnode;
    a.DrT = (const real *)d_DrT;
    a.DsT = (const real *)d_DsT;
    a.DtT = (const real *)d_DtT;
    a.LIFTT = (const real *)d_LIFTT;
    a.fmask = d_fmask;
    a.nP = pml_n;
    a.shot_stride = mesh.K * 9 * R.Np;
    a.mem_stride = pml_n * 18 * R.Np;
    a.shot_map = mapped ? d_shot_map : nullptr;
    a.shot_step = d_step;
    a.shot_len = d_len;
    a.ftau = (real)flux_tau;
    a.rk_a = dgw::rk_a()[stage];
    a.rk_b = dgw::rk_b()[stage];
    a.dt = dt;
  };
  const int ns = slots > 0 ? slots : nshots;
  hipError_t e;
  if (precision == 64) {
    PmlArgs<double> a;
    fill(a);
    e = launch_pml(R.N, 64, ns, &a, stream);
  } else {
    PmlArgs<float> a;
    fill(a);
    e = launch_pml(R.N, 32, ns, &a, stream);
  }
  if (e != hipSuccess) return hipfail(e, "layer kernel launch");
  if (ev) {
    (void)hipEventRecord(pml_ev[pml_ev_used + 1], stream);
    pml_ev_used += 2;
  }
  return DGW_OK;
}

void dgw_ctx::free_pml() {
  dfree(d_pml_elem);
  dfree(d_pml_prof);
  dfree(d_pml_mem);
  dfree(d_pml_mres);
  d_pml_elem = nullptr;
  d_pml_prof = nullptr;
  d_pml_mem = d_pml_mres = nullptr;
  pml_n = 0;
}

int dgw_ctx::clear_pml(int shot) {
  if (pml_n == 0) return DGW_OK;
  const size_t per = (size_t)pml_n * 18 * R.Np * real_size();
  char *base = (char *)d_pml_mem + (shot < 0 ? 0 : shot * per);
  hipError_t e = hipMemsetAsync(base, 0, shot < 0 ? per * nshots : per, stream);
  if (e != hipSuccess) return hipfail(e, "hipMemsetAsync (layer memory)");
  return DGW_OK;
}

int dgw_ctx::build_graph() {
  invalidate_graph();
  hipGraph_t g;
  hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hipfail(e, "hipStreamBeginCapture");
  int from = cur;
  int rc = DGW_OK;
  for (int s = 0; s < kGraphSteps && rc == DGW_OK; ++s) {
    rc = enqueue_step(from, false);
    from = 1 - from;   // 5 stages flip the buffer an odd number of times
  }
  e = hipStreamEndCapture(stream, &g);
  if (rc) return rc;
  if (e != hipSuccess) return hipfail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&graph_exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return hipfail(e, "hipGraphInstantiate");
  graph_ok = true;
  graph_from = cur;
  graph_slots = slots;
  return DGW_OK;
}

// Launch only the listed shots (strictly increasing ids) from here on; the
// full list restores the uncompacted launches.  The map is uploaded on the
// context's stream and waited for, so the host list may change afterwards.
int dgw_ctx::set_active(const std::vector<int32_t> &active) {
  const bool all = (int)active.size() == nshots;
  const int want = all ? nshots : (int)active.size();
  if (want == slots && all == !mapped && (all || active == h_shot_map)) return DGW_OK;
  invalidate_graph();
  slots = want;
  mapped = !all;
  h_shot_map = active;
  if (all) return DGW_OK;
  if (!d_shot_map) {
    d_shot_map = (int32_t *)dalloc(sizeof(int32_t) * nshots);
    if (!d_shot_map) return fail(DGW_ENOMEM, "device allocation failed (shot map)");
  }
  hipError_t e = hipMemcpyAsync(d_shot_map, active.data(), sizeof(int32_t) * active.size(),
                                hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hipfail(e, "hipMemcpyAsync (shot map)");
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hipfail(e, "hipStreamSynchronize");
  return DGW_OK;
}

// Shots about to step must hold their state in d_q[cur]; a shot that sat
// out earlier steps may have it in the other buffer.
int dgw_ctx::gather_shots_to_cur(const std::vector<int64_t> &adv) {
  const size_t n = (size_t)mesh.K * 9 * R.Np * real_size();
  for (int s = 0; s < nshots; ++s) {
    if (adv[s] <= 0 || loc[s] == cur) continue;
    hipError_t e = hipMemcpyAsync((char *)d_q[cur] + s * n,
                                  (const char *)d_q[loc[s]] + s * n, n,
                                  hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) return hipfail(e, "hipMemcpyAsync D2D");
    loc[s] = cur;
  }
  return DGW_OK;
}

// ------------------------------------------------------------------------
// C ABI

extern "C" {

int dgw_create(int order, int precision, int nshots, void *hip_stream,
               dgw_ctx **out) {
  if (!out) return DGW_EINVAL;
  *out = nullptr;
  if (order < 1 || order > DGW_MAX_ORDER) return DGW_EINVAL;
  if (precision != 64 && precision != 32) return DGW_EINVAL;
  if (nshots < 1 || nshots > 65535) return DGW_EINVAL;
  dgw_ctx *c = new (std::nothrow) dgw_ctx();
  if (!c) return DGW_ENOMEM;
  c->precision = precision;
  c->nshots = nshots;
  c->stream = (hipStream_t)hip_stream;
  if (!build_refelem(order, c->R)) {
    delete c;
    return DGW_EINVAL;
  }
  c->block = default_block(0, order, precision);
  *out = c;
  return DGW_OK;
}

void dgw_destroy(dgw_ctx *c) {
  if (!c) return;
  if (c->device_ready) (void)hipStreamSynchronize(c->stream);
  c->invalidate_graph();
  c->free_adjoint();
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->adj_ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->pml_ev) (void)hipEventDestroy(e);
  std::vector<void *> all = c->owned;
  for (void *p : all) c->dfree(p);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char *dgw_last_error(const dgw_ctx *c) {
  return c ? c->err.c_str() : "null context";
}

int dgw_set_allocator(dgw_ctx *c, void *(*alloc)(size_t, void *),
                      void (*free_)(void *, void *), void *user) {
  if (!c) return DGW_EINVAL;
  if (c->have_mesh) return c->fail(DGW_ESTATE, "allocator must be set before the mesh");
  if ((alloc == nullptr) != (free_ == nullptr))
    return c->fail(DGW_EINVAL, "alloc and free must both be set or both be NULL");
  c->alloc_fn = alloc;
  c->free_fn = free_;
  c->alloc_user = user;
  return DGW_OK;
}

int dgw_set_mesh(dgw_ctx *c, int64_t nvert, const double *vxyz, int64_t K,
                 const int32_t *etov, const int32_t *pid, const int8_t *face_bc) {
  if (!c) return DGW_EINVAL;
  if (c->have_mesh) return c->fail(DGW_ESTATE, "mesh already set");
  if (!vxyz || !etov) return c->fail(DGW_EINVAL, "null mesh array");
  for (int64_t i = 0; i < 3 * nvert; ++i)
    if (!std::isfinite(vxyz[i])) return c->fail(DGW_EINVAL, "non-finite vertex");
  if (pid)
    for (int64_t i = 0; i < nvert; ++i)
      if (pid[i] < 0) return c->fail(DGW_EINVAL, "negative periodic id");
  std::string why = build_mesh(c->R, nvert, vxyz, K, etov, pid, face_bc, c->mesh);
  if (!why.empty()) {
    c->mesh = MeshData();
    return c->fail(DGW_EMESH, why);
  }
  int rc;
  if ((rc = c->ensure_device())) return rc;
  c->d_meta = (double *)c->dalloc(sizeof(double) * c->mesh.geo.size());
  c->d_conn = (int32_t *)c->dalloc(sizeof(int32_t) * c->mesh.conn.size());
  c->d_nbtab = (int32_t *)c->dalloc(sizeof(int32_t) * c->mesh.nbtab.size());
  c->d_nbnode = (uint8_t *)c->dalloc(c->mesh.nbnode.size());
  c->d_nbfnode = (uint8_t *)c->dalloc(c->mesh.nbfnode.size());
  if (!c->d_meta || !c->d_conn || !c->d_nbtab || !c->d_nbnode || !c->d_nbfnode)
    return c->fail(DGW_ENOMEM, "device allocation failed (mesh)");
  if ((rc = c->upload(c->d_meta, c->mesh.geo.data(), sizeof(double) * c->mesh.geo.size()))) return rc;
  if ((rc = c->upload(c->d_conn, c->mesh.conn.data(), sizeof(int32_t) * c->mesh.conn.size()))) return rc;
  if ((rc = c->upload(c->d_nbtab, c->mesh.nbtab.data(), sizeof(int32_t) * c->mesh.nbtab.size()))) return rc;
  if ((rc = c->upload(c->d_nbnode, c->mesh.nbnode.data(), c->mesh.nbnode.size()))) return rc;
  if ((rc = c->upload(c->d_nbfnode, c->mesh.nbfnode.data(), c->mesh.nbfnode.size())))
    return rc;
  if ((rc = c->upload_operators())) return rc;
  if ((rc = c->alloc_shots())) return rc;
  c->have_mesh = true;
  return DGW_OK;
}

int dgw_set_material(dgw_ctx *c, const double *rho, const double *lam,
                     const double *mu) {
  if (!c) return DGW_EINVAL;
  if (!c->have_mesh) return c->fail(DGW_ESTATE, "set the mesh first");
  if (!rho || !lam || !mu) return c->fail(DGW_EINVAL, "null material array");
  const int64_t K = c->mesh.K;
  for (int64_t k = 0; k < K; ++k) {
    if (!std::isfinite(rho[k]) || !std::isfinite(lam[k]) || !std::isfinite(mu[k]))
      return c->fail(DGW_EINVAL, "non-finite material at element " + std::to_string(k));
    if (!(rho[k] > 0)) return c->fail(DGW_EINVAL, "rho <= 0 at element " + std::to_string(k));
    if (!(mu[k] >= 0)) return c->fail(DGW_EINVAL, "mu < 0 at element " + std::to_string(k));
    if (!(lam[k] + 2.0 * mu[k] / 3.0 > 0))
      return c->fail(DGW_EINVAL, "lambda + 2 mu / 3 <= 0 at element " + std::to_string(k));
  }
  c->rho.assign(rho, rho + K);
  c->lam.assign(lam, lam + K);
  c->mu.assign(mu, mu + K);
  int rc = c->material_meta();
  if (rc) return rc;
  c->have_mat = true;
  c->touch();
  // the impedance matrices of anisotropic elements depend on rho
  if (c->have_aniso && (rc = c->aniso_table())) return rc;
  return DGW_OK;
}

int dgw_suggest_dt(const dgw_ctx *c, double cfl, double *dt_out) {
  if (!c || !dt_out) return DGW_EINVAL;
  if (!c->have_mesh || !c->have_mat) return DGW_ESTATE;
  if (!(cfl > 0) || !std::isfinite(cfl)) return DGW_EINVAL;
  double best = std::numeric_limits<double>::infinity();
  for (int64_t k = 0; k < c->mesh.K; ++k) {
    double asum = 0;
    for (int f = 0; f < 4; ++f) asum += c->mesh.area[4 * k + f];
    const double rin = 3.0 * c->mesh.volume[k] / asum;
    const double cp = c->have_aniso ? std::sqrt(c->aniso_max_speed2(k))
                                    : std::sqrt((c->lam[k] + 2.0 * c->mu[k]) / c->rho[k]);
    best = std::min(best, rin / cp);
  }
  const int N = c->R.N;
  *dt_out = cfl * 2.0 * best / ((N + 1) * (N + 1));
  return DGW_OK;
}

int dgw_set_dt(dgw_ctx *c, double dt) {
  if (!c) return DGW_EINVAL;
  if (!(dt > 0) || !std::isfinite(dt)) return c->fail(DGW_EINVAL, "dt must be positive");
  c->dt = dt;
  c->have_dt = true;
  c->touch();
  c->invalidate_graph();
  return DGW_OK;
}

int dgw_set_source(dgw_ctx *c, int shot, const double *xyz, const double *moment,
                   double f0, double t0, double amp, int64_t nsteps) {
  if (!c) return DGW_EINVAL;
  if (!c->have_mesh) return c->fail(DGW_ESTATE, "set the mesh first");
  if (shot < 0 || shot >= c->nshots) return c->fail(DGW_ERANGE, "shot out of range");
  if (!xyz) return c->fail(DGW_EINVAL, "null source position");
  if (!std::isfinite(f0) || !std::isfinite(t0) || !std::isfinite(amp) || !(f0 > 0))
    return c->fail(DGW_EINVAL, "invalid Ricker parameters");
  double rst[3];
  const int64_t k = locate_point(c->mesh, xyz, rst);
  if (k < 0) return c->fail(DGW_ERANGE, "source outside the mesh");
  const int Np = c->R.Np;
  std::vector<double> ell(Np);
  eval_basis(c->R, rst, ell.data());
  const double J = c->mesh.geo[k * DGW_META + M_J];
  for (int i = 0; i < Np; ++i) {
    long double s = 0;
    for (int j = 0; j < Np; ++j) s += (long double)c->R.Minv[i * Np + j] * ell[j];
    c->h_src_vec[(size_t)shot * Np + i] = (double)(s / J);
  }
  const double iso[6] = {1, 1, 1, 0, 0, 0};
  const double *mt = moment ? moment : iso;
  for (int i = 0; i < 6; ++i) c->h_src_par[(size_t)shot * 10 + i] = mt[i];
  c->h_src_par[(size_t)shot * 10 + 6] = f0;
  c->h_src_par[(size_t)shot * 10 + 7] = t0;
  c->h_src_par[(size_t)shot * 10 + 8] = amp;
  c->h_src_elem[shot] = (int32_t)k;
  c->h_len[shot] = nsteps > 0 ? nsteps : std::numeric_limits<int64_t>::max();
  c->touch();
  return c->sync_shot_tables();
}

int dgw_set_receivers(dgw_ctx *c, int shot, int nrec, const double *xyz,
                      int64_t max_samples) {
  if (!c) return DGW_EINVAL;
  if (!c->have_mesh) return c->fail(DGW_ESTATE, "set the mesh first");
  if (shot < 0 || shot >= c->nshots) return c->fail(DGW_ERANGE, "shot out of range");
  if (nrec < 0 || nrec > 4096) return c->fail(DGW_ERANGE, "receiver count out of range (0..4096)");
  if (nrec > 0 && !xyz) return c->fail(DGW_EINVAL, "null receiver positions");
  if (max_samples < 0 || max_samples > (int64_t(1) << 31))
    return c->fail(DGW_ERANGE, "trace capacity out of range");
  const int Np = c->R.Np;
  std::vector<int32_t> el(nrec);
  std::vector<double> w((size_t)nrec * Np);
  for (int r = 0; r < nrec; ++r) {
    double rst[3];
    const int64_t k = locate_point(c->mesh, xyz + 3 * r, rst);
    if (k < 0) return c->fail(DGW_ERANGE, "receiver " + std::to_string(r) + " outside the mesh");
    el[r] = (int32_t)k;
    eval_basis(c->R, rst, w.data() + (size_t)r * Np);
  }
  int rc = c->ensure_receivers(std::max(nrec, 1), std::max<int64_t>(max_samples, 1));
  if (rc) return rc;
  for (int r = 0; r < c->rmax; ++r) {
    c->h_rec_elem[(size_t)shot * c->rmax + r] = r < nrec ? el[r] : 0;
    for (int j = 0; j < Np; ++j)
      c->h_rec_w[((size_t)shot * c->rmax + r) * Np + j] = r < nrec ? w[(size_t)r * Np + j] : 0.0;
  }
  c->h_nrec[shot] = nrec;
  c->touch();
  c->h_cap_shot.resize(c->nshots, 0);
  c->h_cap_shot[shot] = max_samples;
  const size_t off = (size_t)shot * c->rmax;
  if ((rc = c->upload(c->d_rec_elem + off, c->h_rec_elem.data() + off, sizeof(int32_t) * c->rmax))) return rc;
  if ((rc = c->upload(c->d_rec_w + off * Np, c->h_rec_w.data() + off * Np, sizeof(double) * c->rmax * Np))) return rc;
  if ((rc = c->upload(c->d_nrec, c->h_nrec.data(), sizeof(int32_t) * c->nshots))) return rc;
  return c->clear_traces(shot);
}

int dgw_set_fields(dgw_ctx *c, int shot, const double *q) {
  if (!c) return DGW_EINVAL;
  if (!c->have_mesh) return c->fail(DGW_ESTATE, "set the mesh first");
  if (shot < 0 || shot >= c->nshots) return c->fail(DGW_ERANGE, "shot out of range");
  if (!q) return c->fail(DGW_EINVAL, "null field array");
  c->touch();
  const size_t n = (size_t)c->mesh.K * 9 * c->R.Np;
  int rc;
  if (c->precision == 64) {
    rc = c->upload((double *)c->d_q[c->cur] + shot * n, q, sizeof(double) * n);
  } else {
    std::vector<float> tmp(q, q + n);
    rc = c->upload((float *)c->d_q[c->cur] + shot * n, tmp.data(), sizeof(float) * n);
  }
  if (rc) return rc;
  if ((rc = c->clear_pml(shot))) return rc;
  if (shot < (int)c->wd_energy.size()) c->wd_energy[shot] = 0.0;
  c->loc[shot] = c->cur;
  c->h_step[shot] = 0;
  if ((rc = c->upload(c->d_step + shot, &c->h_step[shot], sizeof(int64_t)))) return rc;
  return c->clear_traces(shot);
}

int dgw_set_shot_step(dgw_ctx *c, int shot, int64_t step) {
  if (!c) return DGW_EINVAL;
  if (!c->have_mesh) return c->fail(DGW_ESTATE, "set the mesh first");
  if (shot < 0 || shot >= c->nshots) return c->fail(DGW_ERANGE, "shot out of range");
  if (step < 0 || step > c->h_len[shot])
    return c->fail(DGW_ERANGE, "step outside the shot's length");
  c->touch();
  c->h_step[shot] = step;
  return c->upload(c->d_step + shot, &c->h_step[shot], sizeof(int64_t));
}

int dgw_get_fields(dgw_ctx *c, int shot, double *q) {
  if (!c) return DGW_EINVAL;
  if (!c->have_mesh) return c->fail(DGW_ESTATE, "set the mesh first");
  if (shot < 0 || shot >= c->nshots) return c->fail(DGW_ERANGE, "shot out of range");
  if (!q) return c->fail(DGW_EINVAL, "null field array");
  const size_t n = (size_t)c->mesh.K * 9 * c->R.Np;
  const int b = c->loc[shot];
  if (c->precision == 64)
    return c->download(q, (double *)c->d_q[b] + shot * n, sizeof(double) * n);
  std::vector<float> tmp(n);
  int rc = c->download(tmp.data(), (float *)c->d_q[b] + shot * n, sizeof(float) * n);
  if (rc) return rc;
  for (size_t i = 0; i < n; ++i) q[i] = tmp[i];
  return DGW_OK;
}

static int step_core(dgw_ctx *c, int64_t nsteps) {
  if (!c) return DGW_EINVAL;
  if (!c->have_mesh || !c->have_mat || !c->have_dt)
    return c->fail(DGW_ESTATE, "mesh, material and dt must be set before stepping");
  if (nsteps < 0) return c->fail(DGW_EINVAL, "negative step count");
  if (nsteps == 0) return DGW_OK;
  // host mirror of the per-shot counters; capacity check before any work
  int64_t longest = 0;
  std::vector<int64_t> adv(c->nshots);
  for (int s = 0; s < c->nshots; ++s) {
    const int64_t left = c->h_len[s] - c->h_step[s];
    adv[s] = std::max<int64_t>(0, std::min(nsteps, left));
    if (c->h_nrec[s] > 0 && c->h_step[s] + adv[s] > c->h_cap_shot[s])
      return c->fail(DGW_ERANGE, "trace buffer of shot " + std::to_string(s) + " would overflow");
    longest = std::max(longest, adv[s]);
  }
  if (longest == 0) return DGW_OK;
  c->touch();
  int rc;
  if ((rc = c->gather_shots_to_cur(adv))) return rc;
  const int cur0 = c->cur;
  const bool timed = c->timing;
  if (timed) {
    const int need = (int)(10 * longest);
    while ((int)c->ev_pool.size() < need) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) break;
      c->ev_pool.push_back(e);
    }
    c->ev_pool_used = 0;
    const int pneed = c->pml_n > 0 ? need : 0;
    while ((int)c->pml_ev.size() < pneed) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) break;
      c->pml_ev.push_back(e);
    }
    c->pml_ev_used = 0;
  }
  // segments of steps with a fixed set of active shots: a shot advancing
  // adv[s] steps is active in the segments before step adv[s]; each segment
  // launches the blocks of its active shots only
  std::vector<int64_t> ends;
  for (int s = 0; s < c->nshots; ++s)
    if (adv[s] > 0) ends.push_back(adv[s]);
  std::sort(ends.begin(), ends.end());
  ends.erase(std::unique(ends.begin(), ends.end()), ends.end());
  int64_t done = 0;
  for (int64_t end : ends) {
    std::vector<int32_t> active;
    for (int s = 0; s < c->nshots; ++s)
      if (adv[s] >= end) active.push_back(s);
    if ((rc = c->set_active(active))) return rc;
    if (!timed && end - done >= kGraphSteps) {
      if (!c->graph_ok || c->graph_from != c->cur || c->graph_slots != c->slots)
        if ((rc = c->build_graph())) return rc;
      for (; done + kGraphSteps <= end; done += kGraphSteps) {
        hipError_t e = hipGraphLaunch(c->graph_exec, c->stream);
        if (e != hipSuccess) return c->hipfail(e, "hipGraphLaunch");
        // kGraphSteps is even: the buffer roles are unchanged
      }
    }
    for (; done < end; ++done) {
      if ((rc = c->enqueue_step(c->cur, timed))) return rc;
      c->cur = 1 - c->cur;
    }
  }
  for (int s = 0; s < c->nshots; ++s) {
    c->h_step[s] += adv[s];
    if (adv[s] > 0) c->loc[s] = (int)((cur0 + adv[s]) & 1);
  }
  if (timed) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return c->hipfail(e, "hipStreamSynchronize");
    double tot = 0;
    for (int i = 0; i + 1 < c->ev_pool_used; i += 2) {
      float ms = 0;
      (void)hipEventElapsedTime(&ms, c->ev_pool[i], c->ev_pool[i + 1]);
      tot += ms;
    }
    c->timed_launches = c->ev_pool_used / 2;
    c->timed_ms = c->timed_launches ? tot / c->timed_launches : 0.0;
    double ptot = 0;
    for (int i = 0; i + 1 < c->pml_ev_used; i += 2) {
      float ms = 0;
      (void)hipEventElapsedTime(&ms, c->pml_ev[i], c->pml_ev[i + 1]);
      ptot += ms;
    }
    c->pml_timed = c->pml_ev_used / 2;
    c->pml_ms = c->pml_timed ? ptot / c->pml_timed : 0.0;
  }
  return DGW_OK;
}

// The watchdog's check after a chunk of steps: finiteness of every shot's
// fields, then (with a growth bound) each shot's energy against its last.
int dgw_ctx::watchdog_check() {
  if (!d_flag) {
    d_flag = (int *)dalloc(sizeof(int));
    if (!d_flag) return fail(DGW_ENOMEM, "device allocation failed");
  }
  const int64_t n = mesh.K * 9 * R.Np;
  for (int s = 0; s < nshots; ++s) {
    int zero = 0, flag = 0, rc;
    if ((rc = upload(d_flag, &zero, sizeof(int)))) return rc;
    const char *q = (const char *)d_q[loc[s]] + s * n * real_size();
    hipError_t e = launch_finite(precision, q, n, d_flag, stream);
    if (e != hipSuccess) return hipfail(e, "finite kernel launch");
    if ((rc = download(&flag, d_flag, sizeof(int)))) return rc;
    if (flag)
      return fail(DGW_ENONFINITE, "non-finite field value in shot " + std::to_string(s) +
                                      " at step " + std::to_string(h_step[s]));
  }
  if (wd_growth <= 0) return DGW_OK;
  if ((int)wd_energy.size() != nshots) wd_energy.assign(nshots, 0.0);
  for (int s = 0; s < nshots; ++s) {
    double E = 0;
    const int rc = dgw_energy(this, s, &E);
    if (rc) return rc;
    if (wd_energy[s] > 0 && E > wd_growth * wd_energy[s]) {
      char buf[160];
      snprintf(buf, sizeof buf, "energy of shot %d grew by a factor %.3g by step %lld", s,
               E / wd_energy[s], (long long)h_step[s]);
      wd_energy[s] = E;
      return fail(DGW_EGROWTH, buf);
    }
    wd_energy[s] = E;
  }
  return DGW_OK;
}

int dgw_step(dgw_ctx *c, int64_t nsteps) {
  if (!c) return DGW_EINVAL;
  RoctxRange range("dgw_step");
  int rc = DGW_OK;
  if (c->wd_every <= 0 || nsteps <= 0) {
    rc = step_core(c, nsteps);
  } else {
    // chunks ending where the watchdog checks; every chunk is an ordinary
    // call, so the steps are the same as in one call
    int64_t done = 0;
    while (done < nsteps && rc == DGW_OK) {
      const int64_t chunk = std::min(nsteps - done, c->wd_every - c->wd_since);
      rc = step_core(c, chunk);
      if (rc) break;
      done += chunk;
      c->wd_since += chunk;
      if (c->wd_since >= c->wd_every) {
        c->wd_since = 0;
        rc = c->watchdog_check();
      }
    }
  }
  return rc;
}

int dgw_set_watchdog(dgw_ctx *c, int64_t every, double max_growth) {
  if (!c) return DGW_EINVAL;
  if (every < 0) return c->fail(DGW_EINVAL, "negative watchdog interval");
  if (!std::isfinite(max_growth) || max_growth < 0 || (max_growth > 0 && max_growth < 1))
    return c->fail(DGW_EINVAL, "watchdog growth bound must be 0 or a finite value >= 1");
  c->wd_every = every;
  c->wd_growth = max_growth;
  c->wd_since = 0;
  c->wd_energy.assign(c->nshots, 0.0);
  return DGW_OK;
}

int dgw_read_traces(dgw_ctx *c, int shot, double *out, int64_t capacity, int64_t *n) {
  if (!c) return DGW_EINVAL;
  if (!c->have_mesh) return c->fail(DGW_ESTATE, "set the mesh first");
  if (shot < 0 || shot >= c->nshots) return c->fail(DGW_ERANGE, "shot out of range");
  const int nr = c->h_nrec[shot];
  const int64_t have = std::min<int64_t>(c->h_step[shot], c->h_cap_shot.empty() ? 0 : c->h_cap_shot[shot]);
  if (n) *n = nr > 0 ? have : 0;
  if (nr == 0 || !out) return DGW_OK;
  if (capacity < have) return c->fail(DGW_ERANGE, "output capacity smaller than the recorded samples");
  std::vector<double> buf((size_t)c->rmax * 3 * c->cap);
  int rc = c->download(buf.data(), c->d_trace + (size_t)shot * c->rmax * 3 * c->cap,
                       sizeof(double) * buf.size());
  if (rc) return rc;
  for (int r = 0; r < nr; ++r)
    for (int cc = 0; cc < 3; ++cc)
      for (int64_t t = 0; t < have; ++t)
        out[((size_t)r * 3 + cc) * capacity + t] = buf[((size_t)r * 3 + cc) * c->cap + t];
  return DGW_OK;
}

int dgw_shot_steps(dgw_ctx *c, int shot, int64_t *steps) {
  if (!c || !steps) return DGW_EINVAL;
  if (!c->have_mesh) return c->fail(DGW_ESTATE, "set the mesh first");
  if (shot < 0 || shot >= c->nshots) return c->fail(DGW_ERANGE, "shot out of range");
  *steps = c->h_step[shot];
  return DGW_OK;
}

int dgw_energy(dgw_ctx *c, int shot, double *E) {
  if (!c || !E) return DGW_EINVAL;
  if (!c->have_mesh || !c->have_mat) return c->fail(DGW_ESTATE, "mesh and material required");
  if (shot < 0 || shot >= c->nshots) return c->fail(DGW_ERANGE, "shot out of range");
  const int nb = 512;
  if (!c->d_partial) {
    c->d_partial = (double *)c->dalloc(sizeof(double) * nb);
    if (!c->d_partial) return c->fail(DGW_ENOMEM, "device allocation failed");
  }
  const size_t n = (size_t)c->mesh.K * 9 * c->R.Np;
  const char *q = (const char *)c->d_q[c->loc[shot]] + shot * n * c->real_size();
  hipError_t e = launch_energy(c->precision, q, c->mesh.K, c->R.Np, c->d_meta,
                               c->have_aniso ? c->d_aniso : nullptr, c->d_M,
                               c->d_partial, nb, c->stream);
  if (e != hipSuccess) return c->hipfail(e, "energy kernel launch");
  std::vector<double> part(nb);
  int rc = c->download(part.data(), c->d_partial, sizeof(double) * nb);
  if (rc) return rc;
  long double s = 0;
  for (double p : part) s += p;
  *E = (double)s;
  return DGW_OK;
}

int dgw_check_finite(dgw_ctx *c) {
  if (!c) return DGW_EINVAL;
  if (!c->have_mesh) return c->fail(DGW_ESTATE, "set the mesh first");
  if (!c->d_flag) {
    c->d_flag = (int *)c->dalloc(sizeof(int));
    if (!c->d_flag) return c->fail(DGW_ENOMEM, "device allocation failed");
  }
  int zero = 0, flag = 0;
  int rc = c->upload(c->d_flag, &zero, sizeof(int));
  if (rc) return rc;
  const int64_t n = c->mesh.K * 9 * c->R.Np;
  for (int s = 0; s < c->nshots; ++s) {
    const char *q = (const char *)c->d_q[c->loc[s]] + s * n * c->real_size();
    hipError_t e = launch_finite(c->precision, q, n, c->d_flag, c->stream);
    if (e != hipSuccess) return c->hipfail(e, "finite kernel launch");
  }
  if ((rc = c->download(&flag, c->d_flag, sizeof(int)))) return rc;
  if (flag) return c->fail(DGW_ENONFINITE, "non-finite field value");
  return DGW_OK;
}

int dgw_ref_nodes(int order, double *rst) {
  if (order < 1 || order > DGW_MAX_ORDER || !rst) return DGW_EINVAL;
  RefElem R;
  if (!build_refelem(order, R)) return DGW_EINVAL;
  std::memcpy(rst, R.rst.data(), sizeof(double) * R.rst.size());
  return DGW_OK;
}

int dgw_ref_operators(int order, double *Dr, double *Ds, double *Dt, double *M,
                      double *LIFT) {
  if (order < 1 || order > DGW_MAX_ORDER) return DGW_EINVAL;
  RefElem R;
  if (!build_refelem(order, R)) return DGW_EINVAL;
  if (Dr) std::memcpy(Dr, R.Dr.data(), sizeof(double) * R.Dr.size());
  if (Ds) std::memcpy(Ds, R.Ds.data(), sizeof(double) * R.Ds.size());
  if (Dt) std::memcpy(Dt, R.Dt.data(), sizeof(double) * R.Dt.size());
  if (M) std::memcpy(M, R.M.data(), sizeof(double) * R.M.size());
  if (LIFT) std::memcpy(LIFT, R.LIFT.data(), sizeof(double) * R.LIFT.size());
  return DGW_OK;
}

int dgw_set_launch(dgw_ctx *c, int kernel, int elems_per_block, int wgs_per_cu) {
  if (!c) return DGW_EINVAL;
  if (!stage_kernel_supported(kernel, c->R.N, c->precision))
    return c->fail(DGW_EINVAL, "stage kernel not available for this order/precision");
  if (kernel == 2 && c->have_aniso)
    return c->fail(DGW_EINVAL, "stage kernel 2 supports isotropic elements only");
  if (kernel == 2 && wgs_per_cu != 0)
    return c->fail(DGW_EINVAL, "stage kernel 2 runs one work-group per block (wgs_per_cu 0)");
  std::vector<int> ch = stage_block_choices(kernel, c->R.N, c->precision);
  if (elems_per_block == 0) elems_per_block = ch[0];
  if (std::find(ch.begin(), ch.end(), elems_per_block) == ch.end())
    return c->fail(DGW_EINVAL, "unsupported elements-per-block value");
  if (wgs_per_cu < 0 || wgs_per_cu > 64)
    return c->fail(DGW_EINVAL, "work-groups per CU out of range (0..64)");
  c->kernel = kernel;
  c->block = elems_per_block;
  c->wpc = wgs_per_cu;
  c->invalidate_graph();
  return DGW_OK;
}

int dgw_set_damping(dgw_ctx *c, const double *sigma) {
  if (!c) return DGW_EINVAL;
  if (!c->have_mesh) return c->fail(DGW_ESTATE, "set the mesh first");
  c->invalidate_graph();
  c->touch();
  if (!sigma) {
    c->have_sponge = false;
    return DGW_OK;
  }
  const int64_t K = c->mesh.K;
  for (int64_t k = 0; k < K; ++k)
    if (!std::isfinite(sigma[k]) || sigma[k] < 0)
      return c->fail(DGW_EINVAL, "damping rate negative or not finite at element " +
                                     std::to_string(k));
  if (!c->d_sponge) {
    c->d_sponge = (double *)c->dalloc(sizeof(double) * K);
    if (!c->d_sponge) return c->fail(DGW_ENOMEM, "device allocation failed (damping)");
  }
  int rc = c->upload(c->d_sponge, sigma, sizeof(double) * K);
  if (rc) return rc;
  c->have_sponge = true;
  return DGW_OK;
}

int dgw_set_pml(dgw_ctx *c, int64_t n, const int32_t *elements, const double *profile) {
  if (!c) return DGW_EINVAL;
  if (!c->have_mesh) return c->fail(DGW_ESTATE, "set the mesh first");
  if (n < 0) return c->fail(DGW_EINVAL, "negative layer element count");
  const int64_t K = c->mesh.K;
  const int Np = c->R.Np;
  if (n > 0) {
    if (c->have_aniso)
      return c->fail(DGW_ESTATE, "the perfectly matched layer supports isotropic elements only");
    if (!elements || !profile) return c->fail(DGW_EINVAL, "null layer elements or profile");
    if (n > K) return c->fail(DGW_ERANGE, "more layer elements than elements");
    for (int64_t p = 0; p < n; ++p) {
      if (elements[p] < 0 || elements[p] >= K)
        return c->fail(DGW_ERANGE, "layer element out of range at position " + std::to_string(p));
      if (p > 0 && elements[p] <= elements[p - 1])
        return c->fail(DGW_EINVAL, "layer elements must be strictly increasing");
    }
    for (int64_t i = 0; i < n * 6 * Np; ++i)
      if (!std::isfinite(profile[i]) || profile[i] < 0)
        return c->fail(DGW_EINVAL, "layer profile negative or not finite at layer element " +
                                       std::to_string(i / (6 * Np)));
  }
  int rc;
  if ((rc = c->ensure_device())) return rc;
  c->invalidate_graph();
  c->touch();
  // the stream may still be running layer launches that read the old data
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return c->hipfail(e, "hipStreamSynchronize");
  c->free_pml();
  if (n == 0) return DGW_OK;
  const size_t mbytes = (size_t)n * 18 * Np * c->real_size() * c->nshots;
  c->d_pml_elem = (int32_t *)c->dalloc(sizeof(int32_t) * n);
  c->d_pml_prof = (double *)c->dalloc(sizeof(double) * n * 6 * Np);
  c->d_pml_mem = c->dalloc(mbytes);
  c->d_pml_mres = c->dalloc(mbytes);
  if (!c->d_pml_elem || !c->d_pml_prof || !c->d_pml_mem || !c->d_pml_mres) {
    c->free_pml();
    return c->fail(DGW_ENOMEM, "device allocation failed (layer)");
  }
  c->pml_n = n;
  if ((rc = c->upload(c->d_pml_elem, elements, sizeof(int32_t) * n)) ||
      (rc = c->upload(c->d_pml_prof, profile, sizeof(double) * n * 6 * Np)) ||
      (rc = c->clear_pml(-1))) {
    c->free_pml();
    return rc;
  }
  return DGW_OK;
}

int dgw_get_pml_memory(dgw_ctx *c, int shot, double *out) {
  if (!c) return DGW_EINVAL;
  if (c->pml_n == 0) return c->fail(DGW_ESTATE, "no perfectly matched layer is set");
  if (shot < 0 || shot >= c->nshots) return c->fail(DGW_ERANGE, "shot out of range");
  if (!out) return c->fail(DGW_EINVAL, "null output");
  const size_t n = (size_t)c->pml_n * 18 * c->R.Np;
  if (c->precision == 64)
    return c->download(out, (double *)c->d_pml_mem + shot * n, sizeof(double) * n);
  std::vector<float> tmp(n);
  int rc = c->download(tmp.data(), (float *)c->d_pml_mem + shot * n, sizeof(float) * n);
  if (rc) return rc;
  for (size_t i = 0; i < n; ++i) out[i] = tmp[i];
  return DGW_OK;
}

int dgw_set_pml_memory(dgw_ctx *c, int shot, const double *in) {
  if (!c) return DGW_EINVAL;
  if (c->pml_n == 0) return c->fail(DGW_ESTATE, "no perfectly matched layer is set");
  if (shot < 0 || shot >= c->nshots) return c->fail(DGW_ERANGE, "shot out of range");
  if (!in) return c->fail(DGW_EINVAL, "null input");
  const size_t n = (size_t)c->pml_n * 18 * c->R.Np;
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(in[i])) return c->fail(DGW_EINVAL, "non-finite memory variable");
  c->touch();
  if (c->precision == 64)
    return c->upload((double *)c->d_pml_mem + shot * n, in, sizeof(double) * n);
  std::vector<float> tmp(in, in + n);
  return c->upload((float *)c->d_pml_mem + shot * n, tmp.data(), sizeof(float) * n);
}

int dgw_pml_kernel_ms(dgw_ctx *c, double *ms, int64_t *launches) {
  if (!c || !ms || !launches) return DGW_EINVAL;
  *ms = c->pml_ms;
  *launches = c->pml_timed;
  return DGW_OK;
}

int dgw_set_flux(dgw_ctx *c, double tau) {
  if (!c) return DGW_EINVAL;
  if (!(tau >= 0.0 && tau <= 1.0))
    return c->fail(DGW_EINVAL, "flux weight must lie in [0, 1]");
  c->flux_tau = tau;
  c->invalidate_graph();
  c->touch();
  return DGW_OK;
}

int dgw_enable_timing(dgw_ctx *c, int on) {
  if (!c) return DGW_EINVAL;
  c->timing = on != 0;
  return DGW_OK;
}

int dgw_stage_kernel_ms(dgw_ctx *c, double *ms, int64_t *launches) {
  if (!c || !ms) return DGW_EINVAL;
  *ms = c->timed_ms;
  if (launches) *launches = c->timed_launches;
  return DGW_OK;
}

int dgw_adjoint_stage_ms(dgw_ctx *c, double *ms, int64_t *stages) {
  if (!c || !ms) return DGW_EINVAL;
  *ms = c->adj_ms;
  if (stages) *stages = c->adj_timed;
  return DGW_OK;
}

int dgw_state_generation(const dgw_ctx *c, uint64_t *gen) {
  if (!c || !gen) return DGW_EINVAL;
  *gen = c->gen;
  return DGW_OK;
}

int dgw_sizes(const dgw_ctx *c, int *Np, int *Nfp, int64_t *K) {
  if (!c) return DGW_EINVAL;
  if (Np) *Np = c->R.Np;
  if (Nfp) *Nfp = c->R.Nfp;
  if (K) *K = c->mesh.K;
  return DGW_OK;
}

}  // extern "C"
