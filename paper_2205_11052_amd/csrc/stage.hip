// Fused right-hand side + LSERK stage kernel for gfx950.
//
// Work item: a block of BE consecutive elements of one shot.  The items of
// all shots form one flat list.  The hardware dispatches work-groups to the 8
// XCDs round-robin, so the linear work-group id is remapped to give every XCD
// one contiguous range of items: face neighbours (same element, same cube,
// adjacent cubes) are then mostly processed on the same XCD and their traces
// are L2 hits.  Two launch forms share the item code: one work-group per item,
// or a persistent grid of a multiple of 8 work-groups that loop over the
// items (each work-group stays on one XCD).  They are separate instantiations
// so the one-item form carries no loop.
//
// Per item (256 threads):
//   1. every global read of the item's fields is issued at once: the block's
//      fields q[BE][9][Np] (contiguous in HBM, coalesced) and per-element data
//      go to LDS, and each thread gathers the neighbour traces of its face
//      nodes (the neighbour element from the face connectivity, the node from
//      a per-face-node table, so no load waits on a table lookup) into
//      registers;
//   2. one thread per (element, face node): exact Riemann flux in jump form
//      (optionally blended with the central flux; for anisotropic elements
//      from the face's impedance matrices) from the own trace (LDS) and the
//      neighbour's (registers); six lifted
//      quantities go to LDS: the velocity flux and the velocity change dv,
//      both times Fscale (the stress flux is lambda (n.dv) I + mu (dv n^T +
//      n dv^T), n constant per face, so it is formed after lifting dv);
//   3. one thread per (element, node): reference derivatives of the nine
//      fields with Dr, Ds, Dt, the physical volume terms, + the lifted flux,
//      + point source, then res = a res + dt rhs and q_out = q_in + b res.
// q_in and q_out are distinct buffers (neighbour traces are read from q_in
// while other blocks write q_out); res is element-local and updated in place.
#include <hip/hip_runtime.h>

#include <cmath>

#include "dgw_internal.h"
#include "stage_common.h"

namespace dgw {

namespace {

constexpr int kThreads = 256;
using namespace stagec;

// Phase 3 on the matrix cores.  By linearity the element's metric and
// material factors move to the input side: every right-hand-side component
// is rhs_k = sum_a D_a u_{k,a} + LIFT F_k, with u_{k,a} = sum_m c_{k,a,m}
// q_{f(k,m)} a per-node combination of at most three fields (for example
// u_{vx,a} = (1/rho) sum_b X^-1[a][b] sigma_{xb} and
// u_{sxx,a} = (lambda + 2 mu) X^-1[a][0] vx + lambda X^-1[a][1] vy +
// lambda X^-1[a][2] vz).  So the block's right-hand side is one GEMM,
// rhs[i][(e,k)] = [Dr Ds Dt LIFT][i][.] x [u_r; u_s; u_t; F][.][(e,k)],
// whose operator side is shared by all elements: the operator fragments are
// pre-arranged in HBM in MFMA lane order (L1/L2-resident), the data side is
// formed in registers from the LDS tile.  Each wave owns 16 columns
// (element, field); rows are nodes.  The accumulators go through LDS (the
// flux buffer, dead by then) so that the residual loads, the update and the
// stores run over the block's contiguous span, fully coalesced.
template <int N, typename real, int BE, bool AN>
__device__ __forceinline__ void phase3_mfma(const StageArgs<real> &A, const real *sq,
                                            real *sfl, const double *smeta,
                                            const double *ssig, int nE,
                                            int64_t k0, int shot, int64_t step,
                                            real *qout, real *res, int oz, int tid) {
  using M = Mma<real>;
  using v4 = typename M::v4;
  constexpr int Np = Sz<N>::Np, NF = 4 * Sz<N>::Nfp;
  constexpr int MT = (Np + 15) / 16;        // row tiles of 16 nodes
  constexpr int KS = (Np + 3) / 4;          // k-steps per reference direction
  constexpr int KL = NF / 4;                // k-steps of the lift (4 Nfp % 4 == 0)
  constexpr int NT = (9 * BE + 15) / 16;    // column tiles
  static_assert(9 * Np <= 9 * NF, "the flux buffer holds the right-hand side");
  const int lane = tid & 63, g = lane >> 4;
  const int span = nE * 9 * Np;
  // Streaming at order >= 4: the residual (read and written once per stage)
  // and the FP64 output state move with non-temporal loads and stores, so
  // they do not evict the neighbour traces and operators.  Measured on the
  // order-4 82944-element workload (whose streams exceed the 256 MB
  // last-level cache): FP64 370 -> 351 us, FP32 213 -> 204 us (FP32 keeps
  // its output state cached, which measured faster).  The order-3
  // 24576-element gradient workload fits that cache and ran 5% slower with
  // them, so lower orders keep ordinary accesses.
  constexpr bool kStream = N >= 4;
  const bool first = A.rk_a == 0.0;
  // residual loads of this thread's update items (16-byte vectors over the
  // block's contiguous span), issued first
  using SP = Span16<real>;
  constexpr int UV = (BE * 9 * Np / SP::VW + kThreads - 1) / kThreads;
  const SP sp(shot * A.shot_stride + k0 * 9 * Np, span);
  real *rs = res + k0 * 9 * Np, *qo = qout + k0 * 9 * Np;
  v4 acc[NT > 4 ? 2 : 1][MT];
  int ntl = 0;
  if constexpr (!AN && NT == 8) {
    // eight column tiles: each wave takes tiles w and w + 4 and feeds both
    // from every operator fragment it loads (two MFMA chains per fragment)
    const real *q0v[2], *q1v[2], *q2v[2], *flv[2];
    real cv[2][3][3];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int nt = (tid >> 6) + 4 * h;
      const int col = nt * 16 + (lane & 15);
      const bool cok = col < 9 * nE;
      const int e = cok ? col / 9 : 0, k = cok ? col - 9 * (col / 9) : 0;
      const real *qe = sq + e * 9 * Np;
      const double *gm = smeta + e * DGW_META;
      // the same packed column tables as the one-tile path below
      constexpr uint64_t F0 = 0x001000783ull, F1 = 0x122111648ull, F2 = 0x210222567ull;
      constexpr uint32_t X0 = 0x1a000u, X1 = 0x01555u, X2 = 0x2aaaau;
      constexpr uint32_t S0 = 0x36d2200u, S1 = 0x36d1400u, S2 = 0x490a400u;
      const int f0 = (int)((F0 >> (4 * k)) & 15), f1 = (int)((F1 >> (4 * k)) & 15),
                f2 = (int)((F2 >> (4 * k)) & 15);
      const real ri = (real)gm[M_RHOINV], la = (real)gm[M_LAM], mu = (real)gm[M_MU];
      const real l2 = la + 2 * mu;
      auto fac = [&](uint32_t S) -> real {
        const int id = (int)((S >> (3 * k)) & 7);
        return id == 0 ? ri : id == 1 ? l2 : id == 2 ? la : id == 3 ? mu : (real)0;
      };
      const real s0 = fac(S0), s1 = fac(S1), s2 = fac(S2);
      const int x0 = (int)((X0 >> (2 * k)) & 3), x1 = (int)((X1 >> (2 * k)) & 3),
                x2 = (int)((X2 >> (2 * k)) & 3);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const real r0 = (real)gm[M_XINV + 3 * a], r1 = (real)gm[M_XINV + 3 * a + 1],
                   r2 = (real)gm[M_XINV + 3 * a + 2];
        auto pick = [&](int x) { return x == 0 ? r0 : x == 1 ? r1 : r2; };
        cv[h][a][0] = s0 * pick(x0);
        cv[h][a][1] = s1 * pick(x1);
        cv[h][a][2] = s2 * pick(x2);
      }
      q0v[h] = qe + f0 * Np;
      q1v[h] = qe + f1 * Np;
      q2v[h] = qe + f2 * Np;
      flv[h] = sfl + (e * 9 + k) * NF;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[h][mt] = v4{0, 0, 0, 0};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const real *Ab = A.Avol + (size_t)a * KS * MT * 64 + lane + oz;
      for (int ks = 0; ks < KS; ++ks) {
        const int j = 4 * ks + g, jj = j < Np ? j : Np - 1;
        real b[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const real v = cv[h][a][0] * q0v[h][jj] + cv[h][a][1] * q1v[h][jj] +
                         cv[h][a][2] * q2v[h][jj];
          b[h] = j < Np ? v : (real)0;
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const real af = Ab[(ks * MT + mt) * 64];
          acc[0][mt] = M::mma(af, b[0], acc[0][mt]);
          acc[1][mt] = M::mma(af, b[1], acc[1][mt]);
        }
      }
    }
    const real *Al = A.Alift + lane + oz;
    for (int ks = 0; ks < KL; ++ks) {
      const real b0 = flv[0][4 * ks + g], b1 = flv[1][4 * ks + g];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const real af = Al[(ks * MT + mt) * 64];
        acc[0][mt] = M::mma(af, b0, acc[0][mt]);
        acc[1][mt] = M::mma(af, b1, acc[1][mt]);
      }
    }
  } else
  for (int nt = tid >> 6; nt < NT; nt += kThreads / 64, ++ntl) {
    const int col = nt * 16 + (lane & 15);
    const bool cok = col < 9 * nE;
    const int e = cok ? col / 9 : 0, k = cok ? col - 9 * (col / 9) : 0;
    const real *qe = sq + e * 9 * Np;
    const double *gm = smeta + e * DGW_META;
    // input-side coefficients of this column, c[a][m] = s_m X^-1[a][x_m],
    // with the material factor s_m and the metric column x_m of each of
    // the three combined fields f_m given per component k by packed tables
    // (branch-free: the sixteen lanes of a column tile hold different k):
    //   k = 0..2 (vx, vy, vz):   f = sigma row k, s = 1/rho, x = (0, 1, 2)
    //   k = 3..5 (sxx..szz):      f = (vx, vy, vz), s = lambda + 2 mu on
    //                             x = k - 3, lambda elsewhere, x = (0, 1, 2)
    //   k = 6 (syz): f = (vy, vz), s = mu, x = (2, 1)
    //   k = 7 (sxz): f = (vx, vz), s = mu, x = (2, 0)
    //   k = 8 (sxy): f = (vx, vy), s = mu, x = (1, 0)
    // fields (4 bits per k, m = 0, 1, 2)
    constexpr uint64_t F0 = 0x001000783ull, F1 = 0x122111648ull, F2 = 0x210222567ull;
    // metric columns (2 bits per k) and material factor ids (3 bits per k:
    // 0 1/rho, 1 lambda + 2 mu, 2 lambda, 3 mu, 4 zero)
    constexpr uint32_t X0 = 0x1a000u, X1 = 0x01555u, X2 = 0x2aaaau;
    constexpr uint32_t S0 = 0x36d2200u, S1 = 0x36d1400u, S2 = 0x490a400u;
    int f0 = (int)((F0 >> (4 * k)) & 15), f1 = (int)((F1 >> (4 * k)) & 15),
        f2 = (int)((F2 >> (4 * k)) & 15);
    const real ri = (real)gm[M_RHOINV], la = (real)gm[M_LAM], mu = (real)gm[M_MU];
    const real l2 = la + 2 * mu;
    auto fac = [&](uint32_t S) -> real {
      const int id = (int)((S >> (3 * k)) & 7);
      return id == 0 ? ri : id == 1 ? l2 : id == 2 ? la : id == 3 ? mu : (real)0;
    };
    const real s0 = fac(S0), s1 = fac(S1), s2 = fac(S2);
    const int x0 = (int)((X0 >> (2 * k)) & 3), x1 = (int)((X1 >> (2 * k)) & 3),
              x2 = (int)((X2 >> (2 * k)) & 3);
    real c[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const real r0 = (real)gm[M_XINV + 3 * a], r1 = (real)gm[M_XINV + 3 * a + 1],
                 r2 = (real)gm[M_XINV + 3 * a + 2];
      auto pick = [&](int x) { return x == 0 ? r0 : x == 1 ? r1 : r2; };
      c[a][0] = s0 * pick(x0);
      c[a][1] = s1 * pick(x1);
      c[a][2] = s2 * pick(x2);
    }
    if constexpr (AN) {
      // anisotropic stress rows (k >= 3, Voigt row I = k - 3): the fields
      // are (vx, vy, vz) and c[a][m] = sum_b C[I][voigt(m, b)] X^-1[a][b]
      // (selects, so the column setup stays branch-free)
      const bool st = k >= 3;
      const int I = st ? k - 3 : 0;
      const double *Cu = A.aniso + (k0 + e) * DGW_ANI + A_C;
      real cr[6];
#pragma unroll
      for (int J = 0; J < 6; ++J) {
        const int i = I < J ? I : J, j = I < J ? J : I;   // upper triangle
        cr[J] = (real)Cu[i * (11 - i) / 2 + j];
      }
      constexpr int VG[3][3] = {{0, 5, 4}, {5, 1, 3}, {4, 3, 2}};   // voigt(m, b)
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          real v = 0;
#pragma unroll
          for (int b = 0; b < 3; ++b) v += cr[VG[m][b]] * (real)gm[M_XINV + 3 * a + b];
          c[a][m] = st ? v : c[a][m];
        }
      f0 = st ? 0 : f0;
      f1 = st ? 1 : f1;
      f2 = st ? 2 : f2;
    }
    const real *q0 = qe + f0 * Np, *q1 = qe + f1 * Np, *q2 = qe + f2 * Np;
    v4 *ac = acc[ntl];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) ac[mt] = v4{0, 0, 0, 0};
    // volume: three reference directions, K = Np (padded to a multiple of 4)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const real ca0 = c[a][0], ca1 = c[a][1], ca2 = c[a][2];
      const real *Ab = A.Avol + (size_t)a * KS * MT * 64 + lane + oz;
      for (int ks = 0; ks < KS; ++ks) {
        // rows past Np of the last k-step read a valid node and are zeroed
        // (a select, not a branch, so the direction stays one basic block)
        const int j = 4 * ks + g, jj = j < Np ? j : Np - 1;
        real b = ca0 * q0[jj] + ca1 * q1[jj] + ca2 * q2[jj];
        b = j < Np ? b : (real)0;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) ac[mt] = M::mma(Ab[(ks * MT + mt) * 64], b, ac[mt]);
      }
    }
    // lift: the column's flux on the 4 Nfp face nodes
    const real *fl = sfl + (e * 9 + k) * NF;
    const real *Al = A.Alift + lane + oz;
    for (int ks = 0; ks < KL; ++ks) {
      const real b = fl[4 * ks + g];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) ac[mt] = M::mma(Al[(ks * MT + mt) * 64], b, ac[mt]);
    }
  }
  typename SP::vec rv[UV];
#pragma unroll
  for (int u = 0; u < UV; ++u) {
    const int j = tid + u * kThreads;
    if (!first && j < sp.nv) {
      const typename SP::vec *rp = (const typename SP::vec *)(rs + sp.hd) + j;
      if constexpr (kStream)
        rv[u] = __builtin_nontemporal_load(rp);
      else
        rv[u] = *rp;
    }
    else rv[u] = typename SP::vec{};
  }
  const int tl0 = sp.hd + SP::VW * sp.nv;
  const real rh = (!first && tid < sp.hd) ? rs[tid] : (real)0;
  const real rt = (!first && tid < sp.tl) ? rs[tl0 + tid] : (real)0;
  __syncthreads();   // every wave is done with the flux buffer
  // right-hand side to LDS in the block's (element, field, node) order
  ntl = 0;
  for (int nt = tid >> 6; nt < NT; nt += kThreads / 64, ++ntl) {
    const int col = nt * 16 + (lane & 15);
    if (col < 9 * nE) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * mt + M::row(g, r);
          if (i < Np) sfl[col * Np + i] = acc[ntl][mt][r];
        }
    }
  }
  __syncthreads();
  // point source and LSERK update over the contiguous span
  const real ra = (real)A.rk_a, rb = (real)A.rk_b, rdt = (real)A.dt;
  const int64_t es = (int64_t)A.src_elem[shot] - k0;   // source element in block
  double s = 0.0;
  const double *spar = A.src_par + 10 * shot;
  if (es >= 0 && es < nE) s = ricker_d(((double)step + A.rk_c) * A.dt, spar[6], spar[7], spar[8]);
  auto update = [&](int t, real rold) -> real2v<real> {
    real rhs = sfl[t];
    const int e = t / (9 * Np), ci = t - e * 9 * Np, c = ci / Np, i = ci - c * Np;
    if (e == es && c >= 3) rhs += (real)(s * spar[c - 3] * A.src_vec[shot * Np + i]);
    if (A.sponge) rhs -= (real)ssig[e] * sq[t];
    const real rn = first ? rdt * rhs : ra * rold + rdt * rhs;
    return {rn, sq[t] + rb * rn};
  };
#pragma unroll
  for (int u = 0; u < UV; ++u) {
    const int j = tid + u * kThreads;
    if (j >= sp.nv) continue;
    const int b = sp.hd + SP::VW * j;
    typename SP::vec nr, nq;
#pragma unroll
    for (int l = 0; l < SP::VW; ++l) {
      const real2v<real> o = update(b + l, rv[u][l]);
      nr[l] = o.r;
      nq[l] = o.q;
    }
    if constexpr (kStream) {
      __builtin_nontemporal_store(nr, (typename SP::vec *)(rs + b));
      if constexpr (sizeof(real) == 8)
        __builtin_nontemporal_store(nq, (typename SP::vec *)(qo + b));
      else
        *(typename SP::vec *)(qo + b) = nq;
    } else {
      *(typename SP::vec *)(rs + b) = nr;
      *(typename SP::vec *)(qo + b) = nq;
    }
  }
  if (tid < sp.hd) {
    const real2v<real> o = update(tid, rh);
    if constexpr (kStream)
      __builtin_nontemporal_store(o.r, rs + tid);
    else
      rs[tid] = o.r;
    qo[tid] = o.q;
  }
  if (tid < sp.tl) {
    const real2v<real> o = update(tl0 + tid, rt);
    if constexpr (kStream)
      __builtin_nontemporal_store(o.r, rs + tl0 + tid);
    else
      rs[tl0 + tid] = o.r;
    qo[tl0 + tid] = o.q;
  }
}

// Phase 3 on the vector ALUs: one thread per (element, node).  AN:
// anisotropic elements, whose stress rate is C times the strain rate of the
// volume term plus that of the lifted face terms (N(n_f) times the lifted
// dv of each face), with C from the anisotropic per-element data.
template <int N, typename real, int BE, bool AN>
__device__ __forceinline__ void phase3_nodes(const StageArgs<real> &A, const real *sq,
                                             const real *sfl, const double *smeta,
                                             const double *ssig, int nE, int64_t k0,
                                             int shot, int64_t step,
                                             real *qout, real *res, int oz, int tid) {
  constexpr int Np = Sz<N>::Np, Nfp = Sz<N>::Nfp, NF = 4 * Sz<N>::Nfp;
  constexpr int UJ = Np % 7 == 0 ? 7 : Np % 5 == 0 ? 5 : 4;  // divides Np
  for (int t = tid; t < nE * Np; t += kThreads) {
    const int e = t / Np, i = t - e * Np;
    const real *qe = sq + e * 9 * Np;
    const double *g = smeta + e * DGW_META;
    real dr[9], ds[9], dt[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) dr[c] = ds[c] = dt[c] = (real)0;
    // column i of the transposed operators, walked in chunks of UJ rows:
    // inside a chunk every offset is an immediate
    const real *pr = A.DrT + i + oz, *ps = A.DsT + i + oz, *pt = A.DtT + i + oz;
#pragma unroll 1   // a short chunk loop unrolled would hoist every load
    for (int j0 = 0; j0 < Np; j0 += UJ) {
#pragma unroll
      for (int u = 0; u < UJ; ++u) {
        const real a0 = pr[u * Np], a1 = ps[u * Np], a2 = pt[u * Np];
#pragma unroll
        for (int c = 0; c < 9; ++c) {
          const real v = qe[c * Np + j0 + u];
          dr[c] += a0 * v;
          ds[c] += a1 * v;
          dt[c] += a2 * v;
        }
      }
      pr += UJ * Np;
      ps += UJ * Np;
      pt += UJ * Np;
    }
    const int64_t k = k0 + e;
    // the residual loads are issued here, after the volume loop has freed
    // its registers, so their latency overlaps the lift
    real rold[9];
#pragma unroll
    for (int c = 0; c < 9; ++c)
      rold[c] = (A.rk_a == 0.0) ? (real)0 : res[(k * 9 + c) * Np + i];
    real X[9];
#pragma unroll
    for (int u = 0; u < 9; ++u) X[u] = (real)g[M_XINV + u];
    // d/dx_b of field c
    auto D = [&](int c, int b) -> real {
      return X[b] * dr[c] + X[3 + b] * ds[c] + X[6 + b] * dt[c];
    };
    const real ri = (real)g[M_RHOINV], la = (real)g[M_LAM], mu = (real)g[M_MU];
    real rhs[9];
    rhs[0] = (D(3, 0) + D(8, 1) + D(7, 2)) * ri;
    rhs[1] = (D(8, 0) + D(4, 1) + D(6, 2)) * ri;
    rhs[2] = (D(7, 0) + D(6, 1) + D(5, 2)) * ri;
    // anisotropic: the Voigt strain rate (engineering shears), times C below
    real ev[6];
    if constexpr (AN) {
      ev[0] = D(0, 0);
      ev[1] = D(1, 1);
      ev[2] = D(2, 2);
      ev[3] = D(1, 2) + D(2, 1);
      ev[4] = D(0, 2) + D(2, 0);
      ev[5] = D(0, 1) + D(1, 0);
    } else {
      const real divv = D(0, 0) + D(1, 1) + D(2, 2);
      rhs[3] = la * divv + 2 * mu * D(0, 0);
      rhs[4] = la * divv + 2 * mu * D(1, 1);
      rhs[5] = la * divv + 2 * mu * D(2, 2);
      rhs[6] = mu * (D(1, 2) + D(2, 1));
      rhs[7] = mu * (D(0, 2) + D(2, 0));
      rhs[8] = mu * (D(0, 1) + D(1, 0));
    }
    // lift: velocity flux over all faces; lifted dv per face, then the
    // stress components from it and the face normal
    const real *fle = sfl + e * NF * 6;
    const real *pl = A.LIFTT + i + oz;
    real V0 = 0, V1 = 0, V2 = 0;
#pragma unroll 1   // unrolled, the persistent form hoists too much and spills
    for (int f = 0; f < 4; ++f) {
      real U0 = 0, U1 = 0, U2 = 0;
      // the face's lift entries in chunks of LC, each chunk's loads issued
      // before its first use (one by one, every entry cost a round trip)
      constexpr int LC = Nfp % 7 == 0 ? 7 : Nfp % 5 == 0 ? 5 : Nfp;
#pragma unroll
      for (int m0 = 0; m0 < Nfp; m0 += LC) {
        real l[LC];
#pragma unroll
        for (int u = 0; u < LC; ++u) l[u] = pl[(f * Nfp + m0 + u) * Np];
#pragma unroll
        for (int u = 0; u < LC; ++u) {
          const real *s6 = fle + (f * Nfp + m0 + u) * 6;
          V0 += l[u] * s6[0];
          V1 += l[u] * s6[1];
          V2 += l[u] * s6[2];
          U0 += l[u] * s6[3];
          U1 += l[u] * s6[4];
          U2 += l[u] * s6[5];
        }
      }
      const real nx = (real)g[M_NORMAL + 3 * f], ny = (real)g[M_NORMAL + 3 * f + 1],
                 nz = (real)g[M_NORMAL + 3 * f + 2];
      if constexpr (AN) {
        ev[0] += nx * U0;
        ev[1] += ny * U1;
        ev[2] += nz * U2;
        ev[3] += nz * U1 + ny * U2;
        ev[4] += nz * U0 + nx * U2;
        ev[5] += ny * U0 + nx * U1;
      } else {
        const real nU = nx * U0 + ny * U1 + nz * U2;
        rhs[3] += la * nU + 2 * mu * U0 * nx;
        rhs[4] += la * nU + 2 * mu * U1 * ny;
        rhs[5] += la * nU + 2 * mu * U2 * nz;
        rhs[6] += mu * (U1 * nz + U2 * ny);
        rhs[7] += mu * (U0 * nz + U2 * nx);
        rhs[8] += mu * (U0 * ny + U1 * nx);
      }
    }
    rhs[0] += V0;
    rhs[1] += V1;
    rhs[2] += V2;
    if constexpr (AN) {
      // stress rate C ev, C symmetric from its upper triangle
      const double *Cu = A.aniso + k * DGW_ANI + A_C;
      int u = 0;
      real cm[6][6];
#pragma unroll
      for (int a = 0; a < 6; ++a)
#pragma unroll
        for (int b = a; b < 6; ++b) cm[a][b] = cm[b][a] = (real)Cu[u++];
#pragma unroll
      for (int a = 0; a < 6; ++a) {
        real acc = 0;
#pragma unroll
        for (int b = 0; b < 6; ++b) acc += cm[a][b] * ev[b];
        rhs[3 + a] = acc;
      }
    }
    if (A.sponge) {
      const real sg = (real)ssig[e];
#pragma unroll
      for (int c = 0; c < 9; ++c) rhs[c] -= sg * qe[c * Np + i];
    }
    if (A.src_elem[shot] == k) {
      const double *sp = A.src_par + 10 * shot;
      const double s = ricker_d(((double)step + A.rk_c) * A.dt, sp[6], sp[7], sp[8]);
      const double w = s * A.src_vec[shot * Np + i];
#pragma unroll
      for (int c = 0; c < 6; ++c) rhs[3 + c] += (real)(w * sp[c]);
    }
    const real ra = (real)A.rk_a, rb = (real)A.rk_b, rdt = (real)A.dt;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      const int64_t idx = (k * 9 + c) * Np + i;
      // stage 1 (a = 0) never reads res, so stale values cannot leak in
      const real r = (A.rk_a == 0.0) ? rdt * rhs[c] : ra * rold[c] + rdt * rhs[c];
      res[idx] = r;
      qout[idx] = qe[c * Np + i] + rb * r;
    }
  }
}

// Face tables of a block for this thread's face items: the packed
// connectivity code and, for interior faces, the neighbour trace's offset
// in the shot's field array.  Loaded ahead of the gathers (by the persistent
// form one block early).  Both tables are read unconditionally (the index is
// clamped into the block) so every table load is in flight at once.
template <int N, int BE>
struct FaceTab {
  static constexpr int FI = (BE * 4 * Sz<N>::Nfp + kThreads - 1) / kThreads;
  int cn[FI];
  int64_t gb[FI];
  int n1[FI];   // the face node's volume node in its own element
};

template <int N, typename real, int BE>
__device__ __forceinline__ void face_tables(const StageArgs<real> &A, int64_t item,
                                            int64_t nblk, FaceTab<N, BE> &T) {
  constexpr int Np = Sz<N>::Np, Nfp = Sz<N>::Nfp, NF = 4 * Nfp;
  const int slot = (int)(item / nblk);
  const int shot = A.shot_map ? A.shot_map[slot] : slot;
  const int64_t k0 = (item - (int64_t)slot * nblk) * BE;
  const int nE = (int)((A.K - k0) < BE ? (A.K - k0) : BE);
#pragma unroll
  for (int u = 0; u < FaceTab<N, BE>::FI; ++u) {
    const int t = threadIdx.x + u * kThreads;
    const bool ok = k0 < A.K && t < nE * NF;
    const int tt = ok ? t : 0;
    const int e = tt / NF, fm = tt - e * NF, f = fm / Nfp;
    const int64_t k = ok ? k0 + e : 0;
    const int cn = A.conn[k * 4 + f];
    const int nb = A.nbnode[k * NF + fm];
    T.cn[u] = ok ? cn : CONN_ABSORB;
    T.n1[u] = A.fmask[fm];
    // masked arithmetic rather than a select, so the compiler keeps the
    // node-table load unconditional (not behind a wait for cn)
    const int64_t live = -(int64_t)(ok && cn >= 0);
    T.gb[u] = ((int64_t)(cn >> 5) * 9 * Np + nb) & live;
  }
}

// The block's own fields (16-byte vectors over its contiguous span, scalar
// head and tail) and per-element data, loaded into registers: every load is
// issued before any is waited for.
template <int N, typename real, int BE>
struct BlockLoad {
  using SP = Span16<real>;
  static constexpr int QV = (BE * 9 * Sz<N>::Np / SP::VW + kThreads - 1) / kThreads;
  static constexpr int MV = (BE * DGW_META / 2 + kThreads - 1) / kThreads;
  typename SP::vec q[QV];
  real qh, qt;
  double2 m[MV];
  double sg;   // damping rate of element tid of the block (threads < BE)
};

template <int N, typename real, int BE>
__device__ __forceinline__ void block_loads(const StageArgs<real> &A, int64_t item,
                                            int64_t nblk, BlockLoad<N, real, BE> &B) {
  constexpr int Np = Sz<N>::Np;
  using BL = BlockLoad<N, real, BE>;
  using SP = typename BL::SP;
  const int slot = (int)(item / nblk);
  const int shot = A.shot_map ? A.shot_map[slot] : slot;
  const int64_t k0 = (item - (int64_t)slot * nblk) * BE;
  const int nE = (int)((A.K - k0) < BE ? (A.K - k0) : BE);
  const int tid = threadIdx.x;
  // every load is unconditional, with out-of-range lanes clamped to an
  // in-bounds index (their values are never stored): a load under a branch
  // makes the compiler's wait counting conservative, and the neighbour
  // gathers would wait for these loads
  const bool ok = k0 < A.K;
  const int64_t off = ok ? shot * A.shot_stride + k0 * 9 * Np : 0;
  const SP sp(off, ok ? nE * 9 * Np : 1);
  const real *src = A.q_in + off;
  const int nv1 = sp.nv > 0 ? sp.nv - 1 : 0;
  const typename SP::vec *sv = (const typename SP::vec *)(src + sp.hd);
#pragma unroll
  for (int u = 0; u < BL::QV; ++u) {
    const int j = tid + u * kThreads;
    B.q[u] = sv[j < sp.nv ? j : nv1];
  }
  B.qh = src[tid < sp.hd ? tid : 0];
  B.qt = src[tid < sp.tl ? sp.hd + SP::VW * sp.nv + tid : 0];
  const double2 *mv = (const double2 *)(A.meta + (ok ? k0 : 0) * DGW_META);
#pragma unroll
  for (int u = 0; u < BL::MV; ++u) {
    const int j = tid + u * kThreads;
    B.m[u] = mv[j < nE * DGW_META / 2 ? j : 0];
  }
  // the sponge rate: read unconditionally (from the per-element data when
  // there is no sponge, then discarded)
  const double *sgp = A.sponge ? A.sponge : A.meta;
  const double sgv = sgp[(ok ? k0 : 0) + (tid < nE ? tid : 0)];
  B.sg = A.sponge ? sgv : 0.0;
}

template <int N, typename real, int BE, int V>
__device__ __forceinline__ void stage_item(const StageArgs<real> &A, int64_t item,
                                           int64_t nblk, const FaceTab<N, BE> &T,
                                           const BlockLoad<N, real, BE> &B) {
  constexpr int Np = Sz<N>::Np, Nfp = Sz<N>::Nfp, NF = 4 * Sz<N>::Nfp;
  constexpr int FI = (BE * NF + kThreads - 1) / kThreads;   // face items per thread
  // declared here (not passed in) so every access stays an LDS access
  __shared__ real sq[BE * 9 * Np];
  __shared__ __attribute__((aligned(16))) real sfl[BE * NF * (V == 1 || V == 3 ? 9 : 6)];
  __shared__ double smeta[BE * DGW_META];
  __shared__ double ssig[BE];
  const int slot = (int)(item / nblk);
  const int shot = A.shot_map ? A.shot_map[slot] : slot;
  const int64_t step = A.shot_step[shot];
  if (step >= A.shot_len[shot]) return;            // uniform per work-group
  const int64_t k0 = (item - (int64_t)slot * nblk) * BE;
  // never taken (items cover the mesh exactly), but it bounds nE to
  // [1, BE] for the compiler, which keeps the register count low
  if (k0 >= A.K) return;
  const int nE = (int)((A.K - k0) < BE ? (A.K - k0) : BE);
  const real *__restrict__ qin = A.q_in + shot * A.shot_stride;
  real *__restrict__ qout = A.q_out + shot * A.shot_stride;
  real *__restrict__ res = A.res + shot * A.shot_stride;
  const int tid = threadIdx.x;
  // an opaque zero added to the operator addresses: in the persistent form
  // the compiler would otherwise hoist every operator load (they depend on
  // the thread only) out of the item loop, far beyond the register file
  int oz;
  asm volatile("v_mov_b32 %0, 0" : "=v"(oz));

  // ---- 1. all global reads of the item's fields are in flight together ----
  // neighbour traces of this thread's face nodes go to registers; read
  // unconditionally (boundary and idle face items have offset 0, an
  // in-bounds read of the first element that is never used), so no branch
  // makes the compiler wait on earlier loads
  real qp[FI][9];
  int cnv[FI];
#pragma unroll
  for (int u = 0; u < FI; ++u) {
    cnv[u] = T.cn[u];
#pragma unroll
    for (int c = 0; c < 9; ++c) qp[u][c] = qin[T.gb[u] + c * Np];
  }
  // the block's own fields and per-element data (loads issued by
  // block_loads) to LDS
  {
    using BL = BlockLoad<N, real, BE>;
    using SP = typename BL::SP;
    const SP sp(shot * A.shot_stride + k0 * 9 * Np, nE * 9 * Np);
#pragma unroll
    for (int u = 0; u < BL::QV; ++u) {
      const int j = tid + u * kThreads;
      if (j < sp.nv)
#pragma unroll
        for (int l = 0; l < SP::VW; ++l) sq[sp.hd + SP::VW * j + l] = B.q[u][l];
    }
    if (tid < sp.hd) sq[tid] = B.qh;
    if (tid < sp.tl) sq[sp.hd + SP::VW * sp.nv + tid] = B.qt;
#pragma unroll
    for (int u = 0; u < BL::MV; ++u) {
      const int j = tid + u * kThreads;
      if (j < nE * DGW_META / 2) {
        smeta[2 * j] = B.m[u].x;
        smeta[2 * j + 1] = B.m[u].y;
      }
    }
    if (tid < nE) ssig[tid] = B.sg;
  }
  __syncthreads();

  // ---- 2. faces: exact Riemann flux, six lifted quantities per node ----
#pragma unroll
  for (int u = 0; u < FI; ++u) {
    const int t = tid + u * kThreads;
    if (t >= nE * NF) continue;
    const int e = t / NF, fm = t - e * NF, f = fm / Nfp;
    const double *g = smeta + e * DGW_META;
    const real *qe = sq + e * 9 * Np;
    const int n1 = T.n1[u];
    real qm[9], p[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) qm[c] = qe[c * Np + n1];
    const int cn = cnv[u];
    if (cn >= 0) {
#pragma unroll
      for (int c = 0; c < 9; ++c) p[c] = qp[u][c];
    } else if (cn == CONN_FREE) {
#pragma unroll
      for (int c = 0; c < 3; ++c) p[c] = qm[c];
#pragma unroll
      for (int c = 3; c < 9; ++c) p[c] = -qm[c];
    } else {
#pragma unroll
      for (int c = 0; c < 9; ++c) p[c] = (real)0;
    }
    const real nx = (real)g[M_NORMAL + 3 * f], ny = (real)g[M_NORMAL + 3 * f + 1],
               nz = (real)g[M_NORMAL + 3 * f + 2];
    // jumps [v] = v+ - v-, [t] = (sigma+ - sigma-) n
    const real dvx = p[0] - qm[0], dvy = p[1] - qm[1], dvz = p[2] - qm[2];
    const real dsxx = p[3] - qm[3], dsyy = p[4] - qm[4], dszz = p[5] - qm[5];
    const real dsyz = p[6] - qm[6], dsxz = p[7] - qm[7], dsxy = p[8] - qm[8];
    const real dtx = dsxx * nx + dsxy * ny + dsxz * nz;
    const real dty = dsxy * nx + dsyy * ny + dsyz * nz;
    const real dtz = dsxz * nx + dsyz * ny + dszz * nz;
    const real ri = (real)g[M_RHOINV], fs = (real)g[M_FSCALE + f];
    // traction change t* - t- (w) and velocity change dv = v* - v- (u) of
    // the flux states: tu times the exact Riemann states' plus (1 - tu)
    // times the central states' (half the jumps); tu = 1 (upwind) leaves
    // exactly the Riemann terms (1 x + 0 = x)
    const real tu = A.ftau, hc = ((real)1 - tu) * (real)0.5;
    real wx, wy, wz, ux, uy, uz;
    if constexpr (V == 2 || V == 3) {
      // anisotropic: dv = W ([t] + Z+ [v]) and t* - t- = Z- dv with the
      // face's impedance matrices (symmetric 3x3: xx yy zz yz xz xy)
      const double *za = A.aniso + (k0 + e) * DGW_ANI + A_FACE + A_FSTRIDE * f;
      auto smv = [](const double *Z, real x, real y, real z, real (&o)[3]) {
        const real xx = (real)Z[0], yy = (real)Z[1], zz = (real)Z[2], yz = (real)Z[3],
                   xz = (real)Z[4], xy = (real)Z[5];
        o[0] = xx * x + xy * y + xz * z;
        o[1] = xy * x + yy * y + yz * z;
        o[2] = xz * x + yz * y + zz * z;
      };
      real zj[3], dv[3], dtr[3];
      smv(za + A_ZP, dvx, dvy, dvz, zj);
      smv(za + A_W, dtx + zj[0], dty + zj[1], dtz + zj[2], dv);
      smv(za + A_ZM, dv[0], dv[1], dv[2], dtr);
      wx = tu * dtr[0] + hc * dtx;
      wy = tu * dtr[1] + hc * dty;
      wz = tu * dtr[2] + hc * dtz;
      ux = tu * dv[0] + hc * dvx;
      uy = tu * dv[1] + hc * dvy;
      uz = tu * dv[2] + hc * dvz;
    } else {
      const real dvn = dvx * nx + dvy * ny + dvz * nz;
      const real dtn = dtx * nx + dty * ny + dtz * nz;
      const real zp = (real)g[M_ZP], zs = (real)g[M_ZS];
      const real zpn = (real)g[M_ZPNB + f], zsn = (real)g[M_ZSNB + f];
      const real izp = (real)g[M_IZPS + f], izs = (real)g[M_IZSS + f];
      // normal and tangential Riemann amplitudes
      const real kn = (dtn + zpn * dvn) * izp;
      const real kTx = (dtx - dtn * nx + zsn * (dvx - dvn * nx)) * izs;
      const real kTy = (dty - dtn * ny + zsn * (dvy - dvn * ny)) * izs;
      const real kTz = (dtz - dtn * nz + zsn * (dvz - dvn * nz)) * izs;
      wx = tu * (zp * kn * nx + zs * kTx) + hc * dtx;
      wy = tu * (zp * kn * ny + zs * kTy) + hc * dty;
      wz = tu * (zp * kn * nz + zs * kTz) + hc * dtz;
      ux = tu * (kn * nx + kTx) + hc * dvx;
      uy = tu * (kn * ny + kTy) + hc * dvy;
      uz = tu * (kn * nz + kTz) + hc * dvz;
    }
    // velocity flux (t* - t-)/rho and the velocity change dv; the stress
    // flux is lambda (n.dv) I + mu (dv n^T + n dv^T) (anisotropic: C N(n) dv)
    // with n constant on the face, so lifting dv is enough for all six
    // stress components
    if constexpr (V == 0 || V == 2) {
      real *d = sfl + (e * NF + fm) * 6;
      d[0] = fs * wx * ri;
      d[1] = fs * wy * ri;
      d[2] = fs * wz * ri;
      d[3] = fs * ux;
      d[4] = fs * uy;
      d[5] = fs * uz;
    } else {
      // all nine lifted components, field-major (the GEMM's data side)
      const real Dvx = fs * ux, Dvy = fs * uy, Dvz = fs * uz;
      real *d = sfl + e * 9 * NF + fm;
      d[0 * NF] = fs * wx * ri;
      d[1 * NF] = fs * wy * ri;
      d[2 * NF] = fs * wz * ri;
      if constexpr (V == 3) {
        // C N(n) dv
        const real ev[6] = {nx * Dvx, ny * Dvy, nz * Dvz, nz * Dvy + ny * Dvz,
                            nz * Dvx + nx * Dvz, ny * Dvx + nx * Dvy};
        const double *Cu = A.aniso + (k0 + e) * DGW_ANI + A_C;
        real cm[6][6];
        int uu = 0;
#pragma unroll
        for (int a = 0; a < 6; ++a)
#pragma unroll
          for (int b = a; b < 6; ++b) cm[a][b] = cm[b][a] = (real)Cu[uu++];
#pragma unroll
        for (int a = 0; a < 6; ++a) {
          real acc = 0;
#pragma unroll
          for (int b = 0; b < 6; ++b) acc += cm[a][b] * ev[b];
          d[(3 + a) * NF] = acc;
        }
      } else {
        const real la = (real)g[M_LAM], mu = (real)g[M_MU];
        const real ndv = nx * Dvx + ny * Dvy + nz * Dvz;
        d[3 * NF] = la * ndv + 2 * mu * Dvx * nx;
        d[4 * NF] = la * ndv + 2 * mu * Dvy * ny;
        d[5 * NF] = la * ndv + 2 * mu * Dvz * nz;
        d[6 * NF] = mu * (Dvy * nz + Dvz * ny);
        d[7 * NF] = mu * (Dvx * nz + Dvz * nx);
        d[8 * NF] = mu * (Dvx * ny + Dvy * nx);
      }
    }
  }
  __syncthreads();


  if constexpr (V == 1 || V == 3)
    phase3_mfma<N, real, BE, V == 3>(A, sq, sfl, smeta, ssig, nE, k0, shot, step, qout, res,
                                     oz, tid);
  else
    phase3_nodes<N, real, BE, V == 2>(A, sq, sfl, smeta, ssig, nE, k0, shot, step, qout,
                                      res, oz, tid);
}

// One work-group per item.
template <int N, typename real, int BE, int V>
__global__ void __launch_bounds__(kThreads)
stage_kernel(StageArgs<real> A, int64_t nblk, int64_t total) {
  const int64_t item = xcd_item(blockIdx.x, total);
  FaceTab<N, BE> T;
  face_tables<N, real, BE>(A, item, nblk, T);
  BlockLoad<N, real, BE> B;
  block_loads<N, real, BE>(A, item, nblk, B);
  stage_item<N, real, BE, V>(A, item, nblk, T, B);
}

// Persistent grid (a multiple of 8 work-groups) looping over the items;
// the next item's face tables are loaded while the current one is processed.
template <int N, typename real, int BE, int V>
__global__ void __launch_bounds__(kThreads)
stage_kernel_persistent(StageArgs<real> A, int64_t nblk, int64_t total) {
  int64_t L = blockIdx.x;
  FaceTab<N, BE> T;
  if (L < total) face_tables<N, real, BE>(A, xcd_item(L, total), nblk, T);
  for (; L < total; L += gridDim.x) {
    const int64_t item = xcd_item(L, total);
    FaceTab<N, BE> Tn;
    if (L + gridDim.x < total)
      face_tables<N, real, BE>(A, xcd_item(L + gridDim.x, total), nblk, Tn);
    BlockLoad<N, real, BE> B;
    block_loads<N, real, BE>(A, item, nblk, B);
    stage_item<N, real, BE, V>(A, item, nblk, T, B);
    __syncthreads();   // LDS is reused by the next item
    T = Tn;
  }
}

// Elements per work-group for variant V: the largest BE with one thread per
// element node (V = 0: BE * Np <= 256) or one MFMA column per (element,
// field) (V = 1: 9 BE <= 64, four waves of 16 columns), with the LDS tile
// (fields, lifted flux, per-element data) within 64 KB; and half of it.
template <int N, typename real, int V>
struct Shapes {
  static constexpr int Np = Sz<N>::Np, NF = 4 * Sz<N>::Nfp;
  static constexpr int per =
      (9 * Np + (V == 1 || V == 3 ? 9 : 6) * NF) * (int)sizeof(real) + DGW_META * 8;
  static constexpr int cap1 =
      V == 0 || V == 2 ? kThreads / Np : kThreads / 64 * 16 / 9;
  static constexpr int cap2 = 65536 / per;
  static constexpr int a0 = cap1 < cap2 ? cap1 : cap2;
  // matrix-core FP32: two column tiles per wave (14 elements) where the LDS
  // tile fits, and the one-tile block as the second choice (the isotropic
  // form feeds both tiles from each operator fragment, the anisotropic form
  // runs them one after the other); the two share their block choices
  static constexpr bool two = (V == 1 || V == 3) && sizeof(real) == 4 && cap2 >= 2 * cap1;
  static constexpr int a = two ? 2 * cap1 : a0;
  static constexpr int b = two ? cap1 : (a0 / 2 > 0 ? a0 / 2 : 1);
};

template <int N, typename real, int BE, int V>
void launch_be(int64_t grid, bool persistent, int64_t nblk, int64_t total,
               const StageArgs<real> &a, hipStream_t st) {
  if (persistent)
    hipLaunchKernelGGL((stage_kernel_persistent<N, real, BE, V>), dim3((unsigned)grid),
                       dim3(kThreads), 0, st, a, nblk, total);
  else
    hipLaunchKernelGGL((stage_kernel<N, real, BE, V>), dim3((unsigned)grid),
                       dim3(kThreads), 0, st, a, nblk, total);
}

template <int N, typename real, int V>
hipError_t launch_t(int be, int wpc, int ncu, int nshots, const StageArgs<real> &a,
                    hipStream_t st) {
  constexpr int A_ = Shapes<N, real, V>::a, B_ = Shapes<N, real, V>::b;
  if (be != A_ && be != B_) return hipErrorInvalidValue;
  if ((V == 1 || V == 3) && (a.Avol == nullptr || a.Alift == nullptr))
    return hipErrorInvalidValue;
  const int64_t nblk = (a.K + be - 1) / be;
  const int64_t total = nblk * nshots;
  const int64_t pers = ((int64_t)ncu * wpc + 7) / 8 * 8;
  const bool persistent = wpc > 0 && pers < total;
  const int64_t grid = persistent ? pers : total;
  if (be == A_)
    launch_be<N, real, A_, V>(grid, persistent, nblk, total, a, st);
  else
    launch_be<N, real, B_, V>(grid, persistent, nblk, total, a, st);
  return hipGetLastError();
}

template <typename real, int V>
hipError_t launch_r(int N, int be, int wpc, int ncu, int nshots, const void *args,
                    hipStream_t st) {
  const StageArgs<real> &a = *(const StageArgs<real> *)args;
  switch (N) {
    case 1: return launch_t<1, real, V>(be, wpc, ncu, nshots, a, st);
    case 2: return launch_t<2, real, V>(be, wpc, ncu, nshots, a, st);
    case 3: return launch_t<3, real, V>(be, wpc, ncu, nshots, a, st);
    case 4: return launch_t<4, real, V>(be, wpc, ncu, nshots, a, st);
    case 5: return launch_t<5, real, V>(be, wpc, ncu, nshots, a, st);
    case 6: return launch_t<6, real, V>(be, wpc, ncu, nshots, a, st);
  }
  return hipErrorInvalidValue;
}

template <typename real, int V>
std::vector<int> choices_r(int N) {
  switch (N) {
    case 1: return {Shapes<1, real, V>::a, Shapes<1, real, V>::b};
    case 2: return {Shapes<2, real, V>::a, Shapes<2, real, V>::b};
    case 3: return {Shapes<3, real, V>::a, Shapes<3, real, V>::b};
    case 4: return {Shapes<4, real, V>::a, Shapes<4, real, V>::b};
    case 5: return {Shapes<5, real, V>::a, Shapes<5, real, V>::b};
    case 6: return {Shapes<6, real, V>::a, Shapes<6, real, V>::b};
  }
  return {};
}

}  // namespace

hipError_t launch_stage(int kernel, int N, int precision, int be, int wpc, int ncu,
                        int nshots, const void *args, hipStream_t st) {
  if (!stage_kernel_supported(kernel, N, precision)) return hipErrorInvalidValue;
  if (kernel == 2) {
    if (be != stage_split_block() || wpc != 0) return hipErrorInvalidValue;
    return launch_stage_split(N, precision, nshots, args, st);
  }
  // anisotropic elements: instantiations 2 (node per thread) and 3 (matrix
  // cores)
  const bool an = precision == 64 ? ((const StageArgs<double> *)args)->aniso != nullptr
                                  : ((const StageArgs<float> *)args)->aniso != nullptr;
  if (an) {
    if (precision == 64)
      return kernel == 0 ? launch_r<double, 2>(N, be, wpc, ncu, nshots, args, st)
                         : launch_r<double, 3>(N, be, wpc, ncu, nshots, args, st);
    return kernel == 0 ? launch_r<float, 2>(N, be, wpc, ncu, nshots, args, st)
                       : launch_r<float, 3>(N, be, wpc, ncu, nshots, args, st);
  }
  if (precision == 64)
    return kernel == 0 ? launch_r<double, 0>(N, be, wpc, ncu, nshots, args, st)
                       : launch_r<double, 1>(N, be, wpc, ncu, nshots, args, st);
  return kernel == 0 ? launch_r<float, 0>(N, be, wpc, ncu, nshots, args, st)
                     : launch_r<float, 1>(N, be, wpc, ncu, nshots, args, st);
}

bool stage_kernel_supported(int kernel, int N, int precision) {
  if (kernel == 2) return stage_split_supported(N, precision);
  return (kernel == 0 || kernel == 1) && N >= 1 && N <= DGW_MAX_ORDER &&
         (precision == 64 || precision == 32);
}

std::vector<int> stage_block_choices(int kernel, int N, int precision) {
  if (kernel == 2)
    return stage_split_supported(N, precision) ? std::vector<int>{stage_split_block()}
                                               : std::vector<int>{};
  if (kernel == 1) return precision == 64 ? choices_r<double, 1>(N) : choices_r<float, 1>(N);
  if (kernel == 0) return precision == 64 ? choices_r<double, 0>(N) : choices_r<float, 0>(N);
  return {};
}

int default_block(int kernel, int N, int precision) {
  std::vector<int> c = stage_block_choices(kernel, N, precision);
  return c.empty() ? 0 : c[0];
}

}  // namespace dgw
