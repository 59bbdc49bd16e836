// Checkpointed forward run and reverse (adjoint) sweep of the C ABI.
//
// Forward: every shot runs from its (step 0) state for nsteps steps through
// the ordinary stepping path; the state of every shot is copied to a device
// checkpoint every ckpt_every steps; traces are recorded as usual and the
// misfit is reduced on the host in FP64.
// Reverse: segments are visited last to first; a segment is recomputed from
// its checkpoint, storing every step-start state; then for each step, last
// to first: the receiver residual is injected into lam_q, the step's five
// stage inputs are recomputed, and the five stages are reversed (adjoint
// launches).  The gradient accumulates per element in FP64 on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/dgw.h"
#include "dgw_ctx.h"

using namespace dgw;

struct dgw_ctx::Adjoint {
  bool ready = false;
  uint64_t gen = 0;             // context generation the forward ended at
  int64_t nsteps = 0, every = 0;
  std::vector<void *> ckpt;     // per checkpoint: [S][K][9][Np]
  double *d_obs = nullptr;      // [S][rmax][3][nsteps]
  int64_t *d_aux = nullptr;     // per-shot step used by recomputation
  // adjoint operators (row-major D, LIFT) and tables
  void *d_Dr = nullptr, *d_Ds = nullptr, *d_Dt = nullptr, *d_LIFT = nullptr;
  int32_t *d_facepos = nullptr;
};

void dgw_ctx::free_adjoint() {
  if (!adj) return;
  for (void *p : adj->ckpt) dfree(p);
  dfree(adj->d_obs);
  dfree(adj->d_aux);
  dfree(adj->d_Dr);
  dfree(adj->d_Ds);
  dfree(adj->d_Dt);
  dfree(adj->d_LIFT);
  dfree(adj->d_facepos);
  delete adj;
  adj = nullptr;
}

namespace {

template <typename real>
int upload_real(dgw_ctx *c, void **dst, const std::vector<double> &src) {
  std::vector<real> tmp(src.begin(), src.end());
  *dst = c->dalloc(sizeof(real) * tmp.size());
  if (!*dst) return c->fail(DGW_ENOMEM, "device allocation failed (adjoint operators)");
  return c->upload(*dst, tmp.data(), sizeof(real) * tmp.size());
}

int upload_adjoint_tables(dgw_ctx *c) {
  dgw_ctx::Adjoint *a = c->adj;
  if (a->d_Dr) return DGW_OK;
  int rc;
  if (c->precision == 64) {
    if ((rc = upload_real<double>(c, &a->d_Dr, c->R.Dr))) return rc;
    if ((rc = upload_real<double>(c, &a->d_Ds, c->R.Ds))) return rc;
    if ((rc = upload_real<double>(c, &a->d_Dt, c->R.Dt))) return rc;
    if ((rc = upload_real<double>(c, &a->d_LIFT, c->R.LIFT))) return rc;
  } else {
    if ((rc = upload_real<float>(c, &a->d_Dr, c->R.Dr))) return rc;
    if ((rc = upload_real<float>(c, &a->d_Ds, c->R.Ds))) return rc;
    if ((rc = upload_real<float>(c, &a->d_Dt, c->R.Dt))) return rc;
    if ((rc = upload_real<float>(c, &a->d_LIFT, c->R.LIFT))) return rc;
  }
  const int Np = c->R.Np, Nfp = c->R.Nfp;
  std::vector<int32_t> fp(4 * Np, -1);
  for (int f = 0; f < 4; ++f)
    for (int m = 0; m < Nfp; ++m) fp[f * Np + c->R.fmask[f * Nfp + m]] = m;
  a->d_facepos = (int32_t *)c->dalloc(sizeof(int32_t) * fp.size());
  if (!a->d_facepos) return c->fail(DGW_ENOMEM, "device allocation failed (adjoint tables)");
  return c->upload(a->d_facepos, fp.data(), sizeof(int32_t) * fp.size());
}

template <typename real>
void fill_adj(dgw_ctx *c, AdjArgs<real> &a, const void *q, void *lq, void *lr,
              void *zbuf, void *zbuf_next, double *grad, int stage) {
  a.q = (const real *)q;
  a.lam_q = (real *)lq;
  a.lam_r = (real *)lr;
  a.zbuf = (real *)zbuf;
  // stages 4..1 of a step form the lifted adjoint of the next reverse stage
  // (stage - 1); stage 0 is followed by the next step's injection
  a.zbuf_next = (real *)zbuf_next;
  a.lift_next = stage > 0 ? 1 : 0;
  a.next_b = stage > 0 ? rk_b()[stage - 1] : 0.0;
  a.grad = grad;
  a.meta = c->d_meta;
  a.conn = c->d_conn;
  a.nbnode = c->d_nbnode;
  a.nbfnode = c->d_nbfnode;
  a.DrT = (const real *)c->d_DrT;
  a.DsT = (const real *)c->d_DsT;
  a.DtT = (const real *)c->d_DtT;
  a.Dr = (const real *)c->adj->d_Dr;
  a.Ds = (const real *)c->adj->d_Ds;
  a.Dt = (const real *)c->adj->d_Dt;
  a.LIFT = (const real *)c->adj->d_LIFT;
  a.fmask = c->d_fmask;
  a.facepos = c->adj->d_facepos;
  a.sponge = c->have_sponge ? c->d_sponge : nullptr;
  a.K = c->mesh.K;
  a.shot_stride = c->mesh.K * 9 * c->R.Np;
  a.shot_map = nullptr;
  a.shot_step = c->adj->d_aux;
  a.shot_len = c->d_len;
  a.rk_a = rk_a()[stage];
  a.rk_b = rk_b()[stage];
  a.dt = c->dt;
}


// One forward stage of the recomputation over the first `slots` shots of
// `map` (the shots still active at this step).
int stage_explicit(dgw_ctx *c, const void *in, void *out, void *res, int stage,
                   const int32_t *map, int slots) {
  hipError_t e;
  if (c->precision == 64) {
    StageArgs<double> a;
    stage_args(c, a, in, out, res, c->adj->d_aux, stage);
    a.shot_map = map;
    e = launch_stage(c->kernel, c->R.N, 64, c->block, c->wpc, c->ncu, slots, &a, c->stream);
  } else {
    StageArgs<float> a;
    stage_args(c, a, in, out, res, c->adj->d_aux, stage);
    a.shot_map = map;
    e = launch_stage(c->kernel, c->R.N, 32, c->block, c->wpc, c->ncu, slots, &a, c->stream);
  }
  if (e != hipSuccess) return c->hipfail(e, "stage kernel launch (recompute)");
  return DGW_OK;
}

}  // namespace

extern "C" {

int dgw_forward_checkpointed(dgw_ctx *c, int64_t nsteps, int64_t every,
                             const double *d_obs, double *misfit) {
  if (!c) return DGW_EINVAL;
  RoctxRange range("dgw_forward_checkpointed");
  if (!c->have_mesh || !c->have_mat || !c->have_dt)
    return c->fail(DGW_ESTATE, "mesh, material and dt must be set first");
  if (nsteps < 1 || every < 1) return c->fail(DGW_EINVAL, "nsteps and ckpt_every must be >= 1");
  if (!d_obs || !misfit) return c->fail(DGW_EINVAL, "null d_obs or misfit");
  if (c->flux_tau != 1.0)
    return c->fail(DGW_ESTATE, "the adjoint supports the upwind flux only (flux weight 1)");
  if (c->have_aniso)
    return c->fail(DGW_ESTATE, "the adjoint supports isotropic elements only");
  if (c->pml_n > 0)
    return c->fail(DGW_ESTATE, "the adjoint does not support the perfectly matched layer");
  for (int64_t k = 0; k < c->mesh.K; ++k)
    if (c->mu[k] == 0.0)
      return c->fail(DGW_ESTATE, "the gradient is not defined with fluid (mu = 0) elements");
  for (int s = 0; s < c->nshots; ++s) {
    if (c->h_step[s] != 0)
      return c->fail(DGW_ESTATE, "every shot must start at step 0 (set its fields first)");
    const int64_t need = std::min<int64_t>(nsteps, c->h_len[s]);
    if (c->h_nrec[s] > 0 && c->h_cap_shot[s] < need)
      return c->fail(DGW_ERANGE, "trace buffer of shot " + std::to_string(s) +
                                     " is shorter than the run");
  }
  c->free_adjoint();
  c->adj = new dgw_ctx::Adjoint();
  dgw_ctx::Adjoint *a = c->adj;
  a->nsteps = nsteps;
  a->every = every;
  const size_t n = (size_t)c->nshots * c->mesh.K * 9 * c->R.Np * c->real_size();
  const size_t per = (size_t)c->mesh.K * 9 * c->R.Np * c->real_size();
  const int64_t nck = (nsteps + every - 1) / every;
  for (int64_t i = 0; i < nck; ++i) {
    void *p = c->dalloc(n);
    if (!p) {
      c->free_adjoint();
      return c->fail(DGW_ENOMEM, "device allocation failed (checkpoints)");
    }
    a->ckpt.push_back(p);
  }
  int rc;
  for (int64_t i = 0; i < nck; ++i) {
    for (int s = 0; s < c->nshots; ++s) {
      hipError_t e = hipMemcpyAsync((char *)a->ckpt[i] + s * per,
                                    (const char *)c->d_q[c->loc[s]] + s * per, per,
                                    hipMemcpyDeviceToDevice, c->stream);
      if (e != hipSuccess) return c->hipfail(e, "checkpoint copy");
    }
    const int64_t todo = std::min(every, nsteps - i * every);
    if ((rc = dgw_step(c, todo))) return rc;
  }
  // observed data in the device trace layout [S][rmax][3][nsteps]
  const int R = std::max(c->rmax, 1);
  std::vector<double> obs((size_t)c->nshots * R * 3 * nsteps, 0.0);
  int rows = 0;
  for (int s = 0; s < c->nshots; ++s) rows = std::max(rows, c->h_nrec[s]);
  for (int s = 0; s < c->nshots; ++s)
    for (int r = 0; r < c->h_nrec[s]; ++r)
      for (int cc = 0; cc < 3; ++cc)
        std::memcpy(&obs[(((size_t)s * R + r) * 3 + cc) * nsteps],
                    &d_obs[(((size_t)s * rows + r) * 3 + cc) * nsteps],
                    sizeof(double) * nsteps);
  a->d_obs = (double *)c->dalloc(sizeof(double) * obs.size());
  a->d_aux = (int64_t *)c->dalloc(sizeof(int64_t) * c->nshots);
  if (!a->d_obs || !a->d_aux) return c->fail(DGW_ENOMEM, "device allocation failed");
  if ((rc = c->upload(a->d_obs, obs.data(), sizeof(double) * obs.size()))) return rc;
  // misfit per shot from the recorded traces
  for (int s = 0; s < c->nshots; ++s) {
    const int nr = c->h_nrec[s];
    double J = 0.0;
    if (nr > 0) {
      const int64_t have = std::min<int64_t>(nsteps, c->h_len[s]);
      std::vector<double> tr((size_t)nr * 3 * have);
      int64_t got = 0;
      if ((rc = dgw_read_traces(c, s, tr.data(), have, &got))) return rc;
      long double acc = 0;
      for (int r = 0; r < nr; ++r)
        for (int cc = 0; cc < 3; ++cc)
          for (int64_t t = 0; t < have; ++t) {
            const double d = tr[((size_t)r * 3 + cc) * have + t] -
                             obs[(((size_t)s * R + r) * 3 + cc) * nsteps + t];
            acc += (long double)d * d;
          }
      J = (double)(0.5L * c->dt * acc);
    }
    misfit[s] = J;
  }
  a->gen = c->gen;
  a->ready = true;
  return DGW_OK;
}

int dgw_adjoint(dgw_ctx *c, double *g_rho, double *g_lam, double *g_mu) {
  if (!c) return DGW_EINVAL;
  RoctxRange range("dgw_adjoint");
  if (!c->adj || !c->adj->ready)
    return c->fail(DGW_ESTATE, "call dgw_forward_checkpointed first");
  if (c->adj->gen != c->gen)
    return c->fail(DGW_ESTATE, "the solver state changed after dgw_forward_checkpointed "
                               "(a setter, dgw_set_fields or dgw_step ran in between): "
                               "run the checkpointed forward again");
  if (c->flux_tau != 1.0)
    return c->fail(DGW_ESTATE, "the adjoint supports the upwind flux only (flux weight 1)");
  if (c->have_aniso)
    return c->fail(DGW_ESTATE, "the adjoint supports isotropic elements only");
  if (c->pml_n > 0)
    return c->fail(DGW_ESTATE, "the adjoint does not support the perfectly matched layer");
  if (!g_rho || !g_lam || !g_mu) return c->fail(DGW_EINVAL, "null gradient output");
  dgw_ctx::Adjoint *a = c->adj;
  int rc;
  if ((rc = upload_adjoint_tables(c))) return rc;
  const int64_t K = c->mesh.K;
  const int Np = c->R.Np, NF = 4 * c->R.Nfp;
  const size_t rs = c->real_size();
  const size_t n = (size_t)c->nshots * K * 9 * Np * rs;
  std::vector<void *> tmp;
  auto alloc = [&](size_t bytes) -> void * {
    void *p = c->dalloc(bytes);
    if (p) tmp.push_back(p);
    return p;
  };
  auto release = [&]() {
    for (void *p : tmp) c->dfree(p);
    tmp.clear();
  };
  void *lq = alloc(n), *lr = alloc(n), *res = alloc(n);
  // lifted adjoint of the current reverse stage and of the next one
  void *zbuf = alloc((size_t)c->nshots * K * 7 * NF * rs);
  void *zbuf2 = alloc((size_t)c->nshots * K * 7 * NF * rs);
  double *grad = (double *)alloc(sizeof(double) * c->nshots * K * 3);
  // Keep the four inner stage states of every step of a segment when the
  // memory budget allows (every x 4 more states): the segment recompute
  // writes them anyway, and the reverse step then reads them instead of
  // recomputing four stages.  Otherwise only the step-start states are kept.
  size_t budget;
  if (c->adj_budget >= 0) {
    budget = (size_t)c->adj_budget;
  } else {
    size_t fr = 0, tot = 0;
    budget = hipMemGetInfo(&fr, &tot) == hipSuccess ? fr / 4 : 0;
  }
  const bool keep = (size_t)a->every * 4 * n <= budget;
  const int per_step = keep ? 5 : 1;
  auto idx = [&](int64_t sl, int i) { return (size_t)sl * per_step + i; };
  void *st[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  if (!keep)
    for (int i = 1; i < 5; ++i) st[i] = alloc(n);
  std::vector<void *> seg;
  for (int64_t i = 0; i < a->every * per_step; ++i) seg.push_back(alloc(n));
  // the shots by decreasing length: at reverse step s the active shots (those
  // longer than s) are a prefix of this order, so every launch covers just
  // the first nact(s) slots of one map
  std::vector<int32_t> order(c->nshots);
  for (int i = 0; i < c->nshots; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return c->h_len[x] > c->h_len[y]; });
  int32_t *d_order = (int32_t *)alloc(sizeof(int32_t) * c->nshots);
  auto nact = [&](int64_t s) {
    int n_ = 0;
    while (n_ < c->nshots && c->h_len[order[n_]] > s) ++n_;
    return n_;
  };
  bool ok = lq && lr && res && zbuf && zbuf2 && grad && d_order;
  if (!keep) ok = ok && st[1] && st[2] && st[3] && st[4];
  for (void *p : seg) ok = ok && p;
  if (!ok) {
    release();
    return c->fail(DGW_ENOMEM, "device allocation failed (adjoint work space)");
  }
  hipError_t e;
  if ((rc = c->upload(d_order, order.data(), sizeof(int32_t) * c->nshots))) {
    release();
    return rc;
  }
  if ((e = hipMemsetAsync(lq, 0, n, c->stream)) != hipSuccess ||
      (e = hipMemsetAsync(lr, 0, n, c->stream)) != hipSuccess ||
      (e = hipMemsetAsync(res, 0, n, c->stream)) != hipSuccess ||
      (e = hipMemsetAsync(grad, 0, sizeof(double) * c->nshots * K * 3, c->stream)) != hipSuccess) {
    release();
    return c->hipfail(e, "hipMemsetAsync");
  }
  const int64_t nck = (int64_t)a->ckpt.size();
  const int64_t stride = K * 9 * Np;
  // timing: event pairs around the first kAdjTimed reverse stages
  constexpr int kAdjTimed = 200;
  int timed_used = 0;
  if (c->timing)
    while ((int)c->adj_ev.size() < 2 * kAdjTimed) {
      hipEvent_t ev;
      if (hipEventCreate(&ev) != hipSuccess) break;
      c->adj_ev.push_back(ev);
    }
  for (int64_t ci = nck - 1; ci >= 0 && rc == DGW_OK; --ci) {
    const int64_t c0 = ci * a->every;
    const int64_t c1 = std::min(c0 + a->every, a->nsteps);
    e = hipMemcpyAsync(seg[0], a->ckpt[ci], n, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) { rc = c->hipfail(e, "segment restore"); break; }
    // recompute the step-start states of the segment (and, when kept, the
    // inner stage states; the last step's end state is not needed)
    for (int64_t s = c0; s < c1 && rc == DGW_OK; ++s) {
      const bool last = s + 1 == c1;
      if (last && !keep) break;
      if ((e = launch_set_steps(a->d_aux, c->nshots, s, c->stream)) != hipSuccess) {
        rc = c->hipfail(e, "set_steps");
        break;
      }
      const void *in = seg[idx(s - c0, 0)];
      const int na = nact(s);
      for (int i = 0; i < (last ? 4 : 5) && rc == DGW_OK; ++i) {
        void *out = i == 4 ? seg[idx(s - c0 + 1, 0)]
                           : keep ? seg[idx(s - c0, i + 1)] : st[1 + (i & 1)];
        if (na > 0) rc = stage_explicit(c, in, out, res, i, d_order, na);
        in = out;
      }
    }
    for (int64_t s = c1 - 1; s >= c0 && rc == DGW_OK; --s) {
      if ((e = launch_set_steps(a->d_aux, c->nshots, s, c->stream)) != hipSuccess) {
        rc = c->hipfail(e, "set_steps");
        break;
      }
      if (c->rmax > 0 && c->d_trace) {
        e = launch_inject(c->precision, c->nshots, Np, lq, stride, c->d_nrec,
                          c->rmax, c->d_rec_elem, c->d_rec_w, c->d_trace, c->cap,
                          a->d_obs, a->nsteps, a->d_aux, c->d_len, c->dt, c->stream);
        if (e != hipSuccess) { rc = c->hipfail(e, "inject"); break; }
      }
      // stage inputs of step s: kept, or recomputed from the step start
      void *sx[5];
      if (keep) {
        for (int i = 0; i < 5; ++i) sx[i] = seg[idx(s - c0, i)];
      } else {
        sx[0] = seg[idx(s - c0, 0)];
        for (int i = 1; i < 5; ++i) sx[i] = st[i];
        for (int i = 0; i < 4 && rc == DGW_OK; ++i)
          rc = stage_explicit(c, sx[i], sx[i + 1], res, i, d_order, nact(s));
      }
      // the step's first reverse stage lifts w itself (after the
      // injection); each later one reads what the previous main kernel
      // formed, the two buffers alternating
      void *zc = zbuf, *zx = zbuf2;
      const int na = nact(s);
      for (int i = 4; i >= 0 && rc == DGW_OK && na > 0; --i) {
        const bool tm = c->timing && timed_used + 2 <= (int)c->adj_ev.size();
        if (tm) (void)hipEventRecord(c->adj_ev[timed_used], c->stream);
        if (c->precision == 64) {
          AdjArgs<double> aa;
          fill_adj(c, aa, sx[i], lq, lr, zc, zx, grad, i);
          aa.shot_map = d_order;
          e = launch_adjoint_stage(c->R.N, 64, na, &aa, i == 4, c->stream);
        } else {
          AdjArgs<float> aa;
          fill_adj(c, aa, sx[i], lq, lr, zc, zx, grad, i);
          aa.shot_map = d_order;
          e = launch_adjoint_stage(c->R.N, 32, na, &aa, i == 4, c->stream);
        }
        std::swap(zc, zx);
        if (e != hipSuccess) rc = c->hipfail(e, "adjoint stage launch");
        if (tm) {
          (void)hipEventRecord(c->adj_ev[timed_used + 1], c->stream);
          timed_used += 2;
        }
      }
    }
  }
  if (rc == DGW_OK) {
    std::vector<double> g((size_t)c->nshots * K * 3);
    rc = c->download(g.data(), grad, sizeof(double) * g.size());
    if (rc == DGW_OK && c->timing) {
      double tot = 0;
      for (int i = 0; i + 1 < timed_used; i += 2) {
        float ms = 0;
        (void)hipEventElapsedTime(&ms, c->adj_ev[i], c->adj_ev[i + 1]);
        tot += ms;
      }
      c->adj_timed = timed_used / 2;
      c->adj_ms = c->adj_timed ? tot / c->adj_timed : 0.0;
    }
    if (rc == DGW_OK)
      for (int s = 0; s < c->nshots; ++s)
        for (int64_t k = 0; k < K; ++k) {
          g_rho[(size_t)s * K + k] = g[((size_t)s * K + k) * 3 + 0];
          g_lam[(size_t)s * K + k] = g[((size_t)s * K + k) * 3 + 1];
          g_mu[(size_t)s * K + k] = g[((size_t)s * K + k) * 3 + 2];
        }
  } else {
    (void)hipStreamSynchronize(c->stream);
  }
  release();
  return rc;
}

int dgw_set_adjoint_memory(dgw_ctx *c, int64_t bytes) {
  if (!c) return DGW_EINVAL;
  if (bytes < -1) return c->fail(DGW_EINVAL, "adjoint memory budget must be >= -1");
  c->adj_budget = bytes;
  return DGW_OK;
}

}  // extern "C"
