// The library context (opaque to callers of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "dgw_internal.h"

#include <rocprofiler-sdk-roctx/roctx.h>

// A roctx range over a scope (rocprofv3 --marker-trace shows it).
struct RoctxRange {
  explicit RoctxRange(const char *name) { roctxRangePushA(name); }
  ~RoctxRange() { roctxRangePop(); }
  RoctxRange(const RoctxRange &) = delete;
  RoctxRange &operator=(const RoctxRange &) = delete;
};

namespace dgw {
const double *rk_a();
const double *rk_b();
const double *rk_c();
}  // namespace dgw

// Steps per captured HIP graph; even, so the ping-pong buffer roles are the
// same before and after a replay.
constexpr int kGraphSteps = 10;

struct dgw_ctx {
  int precision = 64;
  int nshots = 1;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool device_ready = false;
  int device = 0;                   // HIP device the context's data lives on
  void *(*alloc_fn)(size_t, void *) = nullptr;
  void (*free_fn)(void *, void *) = nullptr;
  void *alloc_user = nullptr;
  std::vector<void *> owned;
  std::string err;

  dgw::RefElem R;
  dgw::MeshData mesh;
  bool have_mesh = false, have_mat = false, have_dt = false;
  double dt = 0;
  double flux_tau = 1.0;            // upwind weight of the face flux
  double *d_sponge = nullptr;       // [K] damping rate (sponge layer)
  bool have_sponge = false;
  std::vector<double> aniso_C;      // [K][21] Voigt stiffness (upper), if set
  double *d_aniso = nullptr;        // [K][DGW_ANI] anisotropic per-element data
  bool have_aniso = false;
  std::vector<double> rho, lam, mu;
  // perfectly matched layer (pml.hip): its elements, per-node profile,
  // memory variables and their stage residual (pml_n = 0: no layer)
  int64_t pml_n = 0;
  int32_t *d_pml_elem = nullptr;
  double *d_pml_prof = nullptr;
  void *d_pml_mem = nullptr, *d_pml_mres = nullptr;

  // device data
  double *d_meta = nullptr;
  int32_t *d_conn = nullptr, *d_nbtab = nullptr, *d_fmask = nullptr;
  uint8_t *d_nbnode = nullptr, *d_nbfnode = nullptr;
  void *d_DrT = nullptr, *d_DsT = nullptr, *d_DtT = nullptr, *d_LIFTT = nullptr;
  void *d_Avol = nullptr, *d_Alift = nullptr;   // MFMA operator fragments
  void *d_Alf = nullptr;                         // per-face lift fragments
  double *d_M = nullptr;
  void *d_q[2] = {nullptr, nullptr};
  void *d_res = nullptr;
  int cur = 0;                      // buffer the next step reads from
  std::vector<int> loc;             // per shot: buffer holding its state
  int64_t *d_step = nullptr, *d_len = nullptr;
  int32_t *d_src_elem = nullptr;
  double *d_src_vec = nullptr, *d_src_par = nullptr;
  std::vector<int64_t> h_step, h_len, h_cap_shot;
  std::vector<int32_t> h_src_elem;
  std::vector<double> h_src_vec, h_src_par;
  int rmax = 0;
  int64_t cap = 0;
  int32_t *d_nrec = nullptr, *d_rec_elem = nullptr;
  double *d_rec_w = nullptr, *d_trace = nullptr;
  std::vector<int32_t> h_nrec, h_rec_elem;
  std::vector<double> h_rec_w;
  double *d_partial = nullptr;
  int *d_flag = nullptr;

  int kernel = 0;                   // stage kernel variant (0: node per thread)
  int block = 0;                    // elements per work-group
  int wpc = 0;                      // persistent work-groups per CU (0: off)
  int ncu = 256;
  hipGraphExec_t graph_exec = nullptr;
  bool graph_ok = false;
  int graph_from = 0;
  // active-shot compaction of dgw_step: while some shots of the batch have
  // finished, the stage and layer launches cover only the active ones,
  // listed in d_shot_map (slots = their count); slots = nshots and no map
  // when every shot is active
  int32_t *d_shot_map = nullptr;
  std::vector<int32_t> h_shot_map;
  int slots = 0;
  bool mapped = false;
  int graph_slots = -1;                // launch slots the graph was captured with

  // Bumped by every call that changes what a run computes (setters,
  // dgw_set_fields, dgw_step); the checkpointed forward records it and the
  // reverse sweep refuses to run when it has moved.
  uint64_t gen = 0;
  void touch() { ++gen; }

  // step watchdog (dgw_set_watchdog): check every wd_every steps, energy
  // bound factor wd_growth (0: finiteness only), steps since the last check,
  // each shot's energy at the last check (0: no baseline)
  int64_t wd_every = 0;
  double wd_growth = 0;
  int64_t wd_since = 0;
  std::vector<double> wd_energy;
  int watchdog_check();

  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  int ev_pool_used = 0;
  double timed_ms = 0;
  int64_t timed_launches = 0;
  // reverse-stage timing (dgw_adjoint with timing on): event pairs around
  // the first reverse stages of the sweep, their average
  std::vector<hipEvent_t> adj_ev;
  double adj_ms = 0;
  int64_t adj_timed = 0;
  // layer-kernel timing (dgw_step with timing on)
  std::vector<hipEvent_t> pml_ev;
  int pml_ev_used = 0;
  double pml_ms = 0;
  int64_t pml_timed = 0;

  // differentiation state (adjoint.cpp)
  struct Adjoint;
  Adjoint *adj = nullptr;
  // device bytes the reverse sweep may spend on kept stage states
  // (-1: a quarter of the free device memory)
  int64_t adj_budget = -1;

  int fail(int code, const std::string &msg);
  int hipfail(hipError_t e, const char *what);
  void *dalloc(size_t bytes);
  void dfree(void *p);
  int ensure_device();
  int upload(void *dst, const void *src, size_t bytes);
  int download(void *dst, const void *src, size_t bytes);
  size_t real_size() const;
  void invalidate_graph();
  int upload_operators();
  int alloc_shots();
  int sync_shot_tables();
  int ensure_receivers(int need_r, int64_t need_cap);
  int clear_traces(int shot);
  int material_meta();
  int aniso_table();                       // anisotropic per-element data
  double aniso_max_speed2(int64_t k) const;  // of an anisotropic element
  int enqueue_step(int from, bool timed);
  int enqueue_pml(const void *in, void *out, int stage, bool timed);
  void free_pml();
  int clear_pml(int shot);                 // zero a shot's memory variables (-1: all)
  int build_graph();
  int gather_shots_to_cur(const std::vector<int64_t> &adv);
  int set_active(const std::vector<int32_t> &active);
  void free_adjoint();
};

// Arguments of one stage launch: state `in` -> `out`, residual `res`, shot
// step counters `steps`, LSERK stage `stage` (0..4).
template <typename real>
inline void stage_args(const dgw_ctx *c, dgw::StageArgs<real> &a, const void *in,
                       void *out, void *res, const int64_t *steps, int stage) {
  a.q_in = (const real *)in;
  a.q_out = (real *)out;
  a.res = (real *)res;
  a.meta = c->d_meta;
  a.conn = c->d_conn;
  a.nbnode = c->d_nbnode;
  a.DrT = (const real *)c->d_DrT;
  a.DsT = (const real *)c->d_DsT;
  a.DtT = (const real *)c->d_DtT;
  a.LIFTT = (const real *)c->d_LIFTT;
  a.Avol = (const real *)c->d_Avol;
  a.Alift = (const real *)c->d_Alift;
  a.Alf = (const real *)c->d_Alf;
  a.fmask = c->d_fmask;
  a.K = c->mesh.K;
  a.shot_stride = c->mesh.K * 9 * c->R.Np;
  a.shot_map = nullptr;
  a.shot_step = steps;
  a.shot_len = c->d_len;
  a.src_elem = c->d_src_elem;
  a.src_vec = c->d_src_vec;
  a.src_par = c->d_src_par;
  a.ftau = (real)c->flux_tau;
  a.sponge = c->have_sponge ? c->d_sponge : nullptr;
  a.aniso = c->have_aniso ? c->d_aniso : nullptr;
  a.rk_a = dgw::rk_a()[stage];
  a.rk_b = dgw::rk_b()[stage];
  a.rk_c = dgw::rk_c()[stage];
  a.dt = c->dt;
}
