// HIP kernels of the discrete adjoint: the exact transpose of one fused
// stage (volume + upwind flux + LIFT) and the parameter gradient
// (d(L q)/d(rho, lambda, mu))^T w, plus receiver-residual injection.
//
// With w the adjoint of a stage's residual (w = lam_r + b lam_q), a reverse
// stage is   lam_q += dt L^T w,   lam_r = a w,   g += dt (d(Lq)/dm)^T w.
// It runs as two launches:
//   adj_lift_kernel: z_f = Fscale_f LIFT_f^T w on every face node (9
//       components), stored per element and face node as the seven
//       combinations the flux transpose uses, with the element's own 1/rho
//       and outward normal: a = z_v / rho (3), c = Zt n (3) with
//       Zt = diag(2 z_xx, 2 z_yy, 2 z_zz) + the off-diagonal z_s, and tr z_s;
//   adj_main_kernel: per face node the transpose of the Riemann flux, taking
//       the own z for the own side and the neighbour's z (at the matched
//       node) for the neighbour's flux, which also depends on this
//       element's trace and impedances; per node the transpose of the
//       volume operator; the gradient from the explicit 1/rho, lambda, mu
//       factors and from the impedances of both sides of every face.
// Within a step the lift kernel runs only for the first reverse stage: each
// main kernel ends by forming the next stage's lifted adjoint from its own
// updated lam_r + b' lam_q (the next stage's w, complete once this stage has
// run, since nothing else touches lam between two stages of a step), into a
// second buffer.  Before a step's first reverse stage the receiver residual
// is injected into lam_q, so that stage lifts afresh.
// Notation (own side "-", neighbour "+", n the own outward normal):
//   [v] = v+ - v-, [t] = (sigma+ - sigma-) n,
//   kn = (n.[t] + Zp+ n.[v]) / (Zp- + Zp+),
//   kT = (P_T [t] + Zs+ P_T [v]) / (Zs- + Zs+),  P_T = I - n n^T,
//   dv = kn n + kT,  dt = Zp- kn n + Zs- kT,
//   flux = (dt / rho, lambda (n.dv) I + mu (dv n^T + n dv^T)).
#include <hip/hip_runtime.h>

#include "dgw_internal.h"

namespace dgw {

namespace {

template <int N>
struct SzA {
  static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  static constexpr int Nfp = (N + 1) * (N + 2) / 2;
};

template <int N>
struct AdjBlock;
template <> struct AdjBlock<1> { static constexpr int be = 16; };
template <> struct AdjBlock<2> { static constexpr int be = 8; };
template <> struct AdjBlock<3> { static constexpr int be = 6; };
template <> struct AdjBlock<4> { static constexpr int be = 4; };
template <> struct AdjBlock<5> { static constexpr int be = 2; };
template <> struct AdjBlock<6> { static constexpr int be = 2; };

constexpr int kT = 256;

// Adjoint of the face flux for one side.  Inputs: n, jumps as seen from this
// side, material of this side (la, mu, zp, zs), impedances of the other side
// (zpo, zso), izp, izs, and the side's lifted adjoint as its seven
// combinations zc = (a = z_v / rho, c = Zt n, tr z_s).
// Outputs: Jv, Jt (adjoint of the jumps [v] and [t]); dZpm, dZpo, dZsm, dZso
// (derivatives of z . flux w.r.t. this side's and the other side's
// impedances); and the forward dv, dt (for the explicit gradient terms).
template <typename real>
__device__ inline void flux_adjoint(
    const real n[3], const real jv[3], const real jt[3], real la,
    real mu, real zp, real zs, real zpo, real zso, real izp, real izs,
    const real zc[7], real Jv[3], real Jt[3], real &dZpm, real &dZpo,
    real &dZsm, real &dZso, real dv[3], real dtr[3]) {
  const real jvn = jv[0] * n[0] + jv[1] * n[1] + jv[2] * n[2];
  const real jtn = jt[0] * n[0] + jt[1] * n[1] + jt[2] * n[2];
  real jvT[3], jtT[3], kTv[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    jvT[a] = jv[a] - jvn * n[a];
    jtT[a] = jt[a] - jtn * n[a];
  }
  const real kn = (jtn + zpo * jvn) * izp;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    kTv[a] = (jtT[a] + zso * jvT[a]) * izs;
    dv[a] = kn * n[a] + kTv[a];
    dtr[a] = zp * kn * n[a] + zs * kTv[a];
  }
  // a = z_v / rho ; b = lambda tr(z_s) n + mu Zt n
  const real trz = zc[6];
  real av[3], bv[3];
  av[0] = zc[0];
  av[1] = zc[1];
  av[2] = zc[2];
  bv[0] = la * trz * n[0] + mu * zc[3];
  bv[1] = la * trz * n[1] + mu * zc[4];
  bv[2] = la * trz * n[2] + mu * zc[5];
  const real an = av[0] * n[0] + av[1] * n[1] + av[2] * n[2];
  const real bn = bv[0] * n[0] + bv[1] * n[1] + bv[2] * n[2];
  const real alpha = bn + zp * an;
  real beta[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) beta[a] = bv[a] + zs * av[a];
  const real betan = beta[0] * n[0] + beta[1] * n[1] + beta[2] * n[2];
  real betaT[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) betaT[a] = beta[a] - betan * n[a];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Jt[a] = izp * alpha * n[a] + izs * betaT[a];
    Jv[a] = zpo * izp * alpha * n[a] + zso * izs * betaT[a];
  }
  const real akT = av[0] * kTv[0] + av[1] * kTv[1] + av[2] * kTv[2];
  const real bkT = betaT[0] * kTv[0] + betaT[1] * kTv[1] + betaT[2] * kTv[2];
  dZpm = an * kn - alpha * kn * izp;
  dZpo = alpha * (jvn - kn) * izp;
  dZsm = akT - izs * bkT;
  dZso = izs * (betaT[0] * (jvT[0] - kTv[0]) + betaT[1] * (jvT[1] - kTv[1]) +
                betaT[2] * (jvT[2] - kTv[2]));
}

template <int N, typename real, int BE>
__global__ void __launch_bounds__(kT) adj_lift_kernel(AdjArgs<real> A) {
  constexpr int Np = SzA<N>::Np, Nfp = SzA<N>::Nfp, NF = 4 * Nfp;
  __shared__ real sw[BE * 9 * Np];
  __shared__ double sfs[BE * 4];
  __shared__ double sgeo[BE * 13];   // 1/rho and the four outward normals
  const int shot = A.shot_map ? A.shot_map[blockIdx.y] : (int)blockIdx.y;
  const int64_t k0 = (int64_t)blockIdx.x * BE;
  if (k0 >= A.K) return;   // never taken (the grid covers the mesh exactly)
  const int nE = (int)((A.K - k0) < BE ? (A.K - k0) : BE);
  const int64_t off = shot * A.shot_stride + k0 * 9 * Np;
  const real b = (real)A.rk_b;
  const int tid = threadIdx.x;
  {
    // w = lam_r + b lam_q over the block's contiguous span (16-byte loads)
    // and Fscale, every load issued (unconditionally, clamped) before any
    // is waited for
    using SP = Span16<real>;
    using vec = typename SP::vec;
    constexpr int QV = (BE * 9 * Np / SP::VW + kT - 1) / kT;
    constexpr int FV = (BE * 4 + kT - 1) / kT;
    const SP sp(off, nE * 9 * Np);
    const real *lr = A.lam_r + off, *lq = A.lam_q + off;
    const int nv1 = sp.nv > 0 ? sp.nv - 1 : 0;
    vec vr[QV], vl[QV];
#pragma unroll
    for (int u = 0; u < QV; ++u) {
      const int j = tid + u * kT, jj = j < sp.nv ? j : nv1;
      vr[u] = ((const vec *)(lr + sp.hd))[jj];
      vl[u] = ((const vec *)(lq + sp.hd))[jj];
    }
    const int ih = tid < sp.hd ? tid : 0;
    const int it = tid < sp.tl ? sp.hd + SP::VW * sp.nv + tid : 0;
    const real hr = lr[ih], hl = lq[ih], tr_ = lr[it], tl_ = lq[it];
    double fsv[FV];
#pragma unroll
    for (int u = 0; u < FV; ++u) {
      const int t = tid + u * kT, tt = t < nE * 4 ? t : 0;
      fsv[u] = A.meta[(k0 + tt / 4) * DGW_META + M_FSCALE + (tt & 3)];
    }
    constexpr int GV = (BE * 13 + kT - 1) / kT;
    double gv[GV];
#pragma unroll
    for (int u = 0; u < GV; ++u) {
      const int t = tid + u * kT, tt = t < nE * 13 ? t : 0;
      const int e = tt / 13, j = tt - 13 * e;
      gv[u] = A.meta[(k0 + e) * DGW_META + (j == 0 ? M_RHOINV : M_NORMAL + j - 1)];
    }
    const int64_t step = A.shot_step[shot];
    if (step >= A.shot_len[shot]) return;   // uniform per work-group
#pragma unroll
    for (int u = 0; u < QV; ++u) {
      const int j = tid + u * kT;
      if (j < sp.nv) {
        const int o = sp.hd + SP::VW * j;
#pragma unroll
        for (int l = 0; l < SP::VW; ++l) sw[o + l] = vr[u][l] + b * vl[u][l];
      }
    }
    if (tid < sp.hd) sw[tid] = hr + b * hl;
    if (tid < sp.tl) sw[it] = tr_ + b * tl_;
#pragma unroll
    for (int u = 0; u < FV; ++u) {
      const int t = tid + u * kT;
      if (t < nE * 4) sfs[t] = fsv[u];
    }
#pragma unroll
    for (int u = 0; u < GV; ++u) {
      const int t = tid + u * kT;
      if (t < nE * 13) sgeo[t] = gv[u];
    }
  }
  __syncthreads();
  real *zb = A.zbuf + (shot * A.K + k0) * 7 * NF;
  for (int t = threadIdx.x; t < nE * NF; t += kT) {
    const int e = t / NF, fm = t - e * NF;
    const real *we = sw + e * 9 * Np;
    real acc[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) acc[c] = 0;
    for (int i = 0; i < Np; ++i) {
      const real l = A.LIFT[i * NF + fm];
#pragma unroll
      for (int c = 0; c < 9; ++c) acc[c] += l * we[c * Np + i];
    }
    const int f = fm / Nfp;
    const real fs = (real)sfs[e * 4 + f];
    real z[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) z[c] = fs * acc[c];
    const double *ge = sgeo + e * 13;
    const real ri = (real)ge[0];
    const real n0 = (real)ge[1 + 3 * f], n1 = (real)ge[2 + 3 * f], n2 = (real)ge[3 + 3 * f];
    real zc[7];
    zc[0] = ri * z[0];
    zc[1] = ri * z[1];
    zc[2] = ri * z[2];
    zc[3] = 2 * z[3] * n0 + z[8] * n1 + z[7] * n2;
    zc[4] = z[8] * n0 + 2 * z[4] * n1 + z[6] * n2;
    zc[5] = z[7] * n0 + z[6] * n1 + 2 * z[5] * n2;
    zc[6] = z[3] + z[4] + z[5];
#pragma unroll
    for (int c = 0; c < 7; ++c) zb[(e * 7 + c) * NF + fm] = zc[c];
  }
}

template <int N, typename real, int BE>
__global__ void __launch_bounds__(kT) adj_main_kernel(AdjArgs<real> A) {
  constexpr int Np = SzA<N>::Np, Nfp = SzA<N>::Nfp, NF = 4 * Nfp;
  __shared__ real sw[BE * 9 * Np];
  __shared__ real sq[BE * 9 * Np];
  __shared__ real sfa[BE * 9 * NF];
  __shared__ double sg[BE * 3 * NF];
  __shared__ double sgv[BE * 3 * Np];
  __shared__ double smeta[BE * DGW_META];

  const int shot = A.shot_map ? A.shot_map[blockIdx.y] : (int)blockIdx.y;
  const int64_t k0 = (int64_t)blockIdx.x * BE;
  if (k0 >= A.K) return;   // never taken (the grid covers the mesh exactly)
  const int nE = (int)((A.K - k0) < BE ? (A.K - k0) : BE);
  const int64_t soff = shot * A.shot_stride;
  const real *__restrict__ q = A.q + soff;
  real *lq = A.lam_q + soff;
  real *lr = A.lam_r + soff;
  const real *zb = A.zbuf + shot * A.K * 7 * NF;
  const real b = (real)A.rk_b;
  const int tid = threadIdx.x;

  // ---- every global read of the block is issued before any is waited
  //      for; all unconditional, with out-of-range lanes clamped to
  //      in-bounds indices (a load under a branch makes the compiler wait on
  //      it, and vmcnt completes loads in order)
  constexpr int FI = (BE * NF + kT - 1) / kT;   // face items per thread
  // level 1: this thread's face tables and own z
  int cnv[FI], n1v[FI], n2v[FI], f2v[FI];
  real zo[FI][7];
#pragma unroll
  for (int u = 0; u < FI; ++u) {
    const int t = tid + u * kT;
    const bool ok = t < nE * NF;
    const int tt = ok ? t : 0;
    const int e = tt / NF, fm = tt - e * NF, f = fm / Nfp;
    const int64_t k = k0 + e;
    const int cn = A.conn[k * 4 + f];
    cnv[u] = ok ? cn : CONN_ABSORB;
    n1v[u] = A.fmask[fm];
    n2v[u] = A.nbnode[k * NF + fm];
    f2v[u] = A.nbfnode[k * NF + fm];
#pragma unroll
    for (int c = 0; c < 7; ++c) zo[u][c] = zb[(k * 7 + c) * NF + fm];
  }
  // the block's w = lam_r + b lam_q and stage input q (16-byte vectors over
  // its contiguous span) and per-element data
  using SP = Span16<real>;
  using vec = typename SP::vec;
  constexpr int QV = (BE * 9 * Np / SP::VW + kT - 1) / kT;
  constexpr int MV = (BE * DGW_META / 2 + kT - 1) / kT;
  const SP sp(soff + k0 * 9 * Np, nE * 9 * Np);
  const real *lrb = lr + k0 * 9 * Np, *lqb = lq + k0 * 9 * Np, *qb = q + k0 * 9 * Np;
  const int nv1 = sp.nv > 0 ? sp.nv - 1 : 0;
  vec vr[QV], vl[QV], vq[QV];
#pragma unroll
  for (int u = 0; u < QV; ++u) {
    const int j = tid + u * kT, jj = j < sp.nv ? j : nv1;
    vr[u] = ((const vec *)(lrb + sp.hd))[jj];
    vl[u] = ((const vec *)(lqb + sp.hd))[jj];
    vq[u] = ((const vec *)(qb + sp.hd))[jj];
  }
  const int ih = tid < sp.hd ? tid : 0;
  const int it = tid < sp.tl ? sp.hd + SP::VW * sp.nv + tid : 0;
  const real hr = lrb[ih], hl = lqb[ih], hq = qb[ih];
  const real tr_ = lrb[it], tl_ = lqb[it], tq = qb[it];
  const double2 *mv = (const double2 *)(A.meta + k0 * DGW_META);
  double2 mm[MV];
#pragma unroll
  for (int u = 0; u < MV; ++u) {
    const int j = tid + u * kT;
    mm[u] = mv[j < nE * DGW_META / 2 ? j : 0];
  }
  const int64_t step = A.shot_step[shot];
  if (step >= A.shot_len[shot]) return;   // uniform per work-group
  // level 2: the neighbour's trace, z at the matched face node and material
  // (element 0 where the face has no neighbour; never used)
  real qp[FI][9], zn[FI][7], gn[FI][4];
#pragma unroll
  for (int u = 0; u < FI; ++u) {
    const int64_t nb = cnv[u] >= 0 ? (int64_t)(cnv[u] >> 5) : 0;
#pragma unroll
    for (int c = 0; c < 9; ++c) qp[u][c] = q[(nb * 9 + c) * Np + n2v[u]];
#pragma unroll
    for (int c = 0; c < 7; ++c) zn[u][c] = zb[(nb * 7 + c) * NF + f2v[u]];
    const double *g2 = A.meta + nb * DGW_META;
    gn[u][0] = (real)g2[M_LAM];
    gn[u][1] = (real)g2[M_MU];
    gn[u][2] = (real)g2[M_ZP];
    gn[u][3] = (real)g2[M_ZS];
  }
  // the block's values to LDS
#pragma unroll
  for (int u = 0; u < QV; ++u) {
    const int j = tid + u * kT;
    if (j < sp.nv) {
      const int o = sp.hd + SP::VW * j;
#pragma unroll
      for (int l = 0; l < SP::VW; ++l) {
        sw[o + l] = vr[u][l] + b * vl[u][l];
        sq[o + l] = vq[u][l];
      }
    }
  }
  if (tid < sp.hd) {
    sw[tid] = hr + b * hl;
    sq[tid] = hq;
  }
  if (tid < sp.tl) {
    sw[it] = tr_ + b * tl_;
    sq[it] = tq;
  }
#pragma unroll
  for (int u = 0; u < MV; ++u) {
    const int j = tid + u * kT;
    if (j < nE * DGW_META / 2) {
      smeta[2 * j] = mm[u].x;
      smeta[2 * j + 1] = mm[u].y;
    }
  }
  __syncthreads();

  // ---- faces: flux transpose and face gradient terms ------------------
#pragma unroll
  for (int u = 0; u < FI; ++u) {
    const int t = tid + u * kT;
    if (t >= nE * NF) continue;
    const int e = t / NF, fm = t - e * NF, f = fm / Nfp;
    const double *g = smeta + e * DGW_META;
    const real *qe = sq + e * 9 * Np;
    const int n1 = n1v[u];
    const int cn = cnv[u];
    real qm[9], qpp[9];
    const real *z = zo[u];
#pragma unroll
    for (int c = 0; c < 9; ++c) qm[c] = qe[c * Np + n1];
    if (cn >= 0) {
#pragma unroll
      for (int c = 0; c < 9; ++c) qpp[c] = qp[u][c];
    } else if (cn == CONN_FREE) {
#pragma unroll
      for (int c = 0; c < 3; ++c) qpp[c] = qm[c];
#pragma unroll
      for (int c = 3; c < 9; ++c) qpp[c] = -qm[c];
    } else {
#pragma unroll
      for (int c = 0; c < 9; ++c) qpp[c] = 0;
    }
    real n[3] = {(real)g[M_NORMAL + 3 * f], (real)g[M_NORMAL + 3 * f + 1],
                 (real)g[M_NORMAL + 3 * f + 2]};
    real jv[3], js[6], jt[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) jv[a] = qpp[a] - qm[a];
#pragma unroll
    for (int a = 0; a < 6; ++a) js[a] = qpp[3 + a] - qm[3 + a];
    jt[0] = js[0] * n[0] + js[5] * n[1] + js[4] * n[2];
    jt[1] = js[5] * n[0] + js[1] * n[1] + js[3] * n[2];
    jt[2] = js[4] * n[0] + js[3] * n[1] + js[2] * n[2];
    const real ri = (real)g[M_RHOINV], la = (real)g[M_LAM], mu = (real)g[M_MU];
    const real zp = (real)g[M_ZP], zs = (real)g[M_ZS];
    const real zpo = (real)g[M_ZPNB + f], zso = (real)g[M_ZSNB + f];
    const real izp = (real)g[M_IZPS + f], izs = (real)g[M_IZSS + f];
    real Jv[3], Jt[3], dv[3], dtr[3], dZpm, dZpo, dZsm, dZso;
    flux_adjoint<real>(n, jv, jt, la, mu, zp, zs, zpo, zso, izp, izs, z,
                       Jv, Jt, dZpm, dZpo, dZsm, dZso, dv, dtr);
    // adjoint of sigma from [t] = [sigma] n (Voigt xx yy zz yz xz xy)
    real Js[6];
    Js[0] = Jt[0] * n[0];
    Js[1] = Jt[1] * n[1];
    Js[2] = Jt[2] * n[2];
    Js[3] = Jt[1] * n[2] + Jt[2] * n[1];
    Js[4] = Jt[0] * n[2] + Jt[2] * n[0];
    Js[5] = Jt[0] * n[1] + Jt[1] * n[0];
    real out[9];
    if (cn == CONN_FREE) {
      // v+ = v-, sigma+ = -sigma-
#pragma unroll
      for (int a = 0; a < 3; ++a) out[a] = 0;
#pragma unroll
      for (int a = 0; a < 6; ++a) out[3 + a] = -2 * Js[a];
    } else {
#pragma unroll
      for (int a = 0; a < 3; ++a) out[a] = -Jv[a];
#pragma unroll
      for (int a = 0; a < 6; ++a) out[3 + a] = -Js[a];
    }
    // explicit material factors of the own flux: with a = z_v / rho,
    // d/d(1/rho) is z_v . dt = rho a . dt (so d/drho is -(1/rho) a . dt),
    // d/dlambda is tr z_s (n . dv), d/dmu is dv . Zt n
    const real ndv = n[0] * dv[0] + n[1] * dv[1] + n[2] * dv[2];
    double gr = -(double)ri * (double)(z[0] * dtr[0] + z[1] * dtr[1] + z[2] * dtr[2]);
    double gl = (double)z[6] * (double)ndv;
    double gm = (double)(z[3] * dv[0] + z[4] * dv[1] + z[5] * dv[2]);
    double dzp = dZpm, dzs = dZsm;
    if (cn < 0) {
      dzp += dZpo;   // boundary: the ghost impedance is the own impedance
      dzs += dZso;
    } else {
      // the neighbour's flux on this face, seen from the neighbour: normal
      // -n, jumps -[v] and [t], its own material, this element as "+"
      real nn[3] = {-n[0], -n[1], -n[2]};
      real jvn[3] = {-jv[0], -jv[1], -jv[2]};
      real Jv2[3], Jt2[3], dv2[3], dt2[3], a1, a2, a3, a4;
      flux_adjoint<real>(nn, jvn, jt, gn[u][0], gn[u][1], gn[u][2], gn[u][3],
                         zp, zs, izp, izs, zn[u], Jv2, Jt2, a1, a2, a3, a4, dv2, dt2);
      // this element is the neighbour's "+" side: [v]' = v_k - v_nb etc.
      out[0] += Jv2[0];
      out[1] += Jv2[1];
      out[2] += Jv2[2];
      out[3] += Jt2[0] * nn[0];
      out[4] += Jt2[1] * nn[1];
      out[5] += Jt2[2] * nn[2];
      out[6] += Jt2[1] * nn[2] + Jt2[2] * nn[1];
      out[7] += Jt2[0] * nn[2] + Jt2[2] * nn[0];
      out[8] += Jt2[0] * nn[1] + Jt2[1] * nn[0];
      dzp += a2;
      dzs += a4;
    }
    real *dst = sfa + e * 9 * NF + fm;
#pragma unroll
    for (int c = 0; c < 9; ++c) dst[c * NF] = out[c];
    // impedance chain rule
    const double rho = g[47], lam = g[M_LAM], muu = g[M_MU];
    const double Zp = g[M_ZP], Zs = g[M_ZS];
    gr += dzp * (lam + 2 * muu) / (2 * Zp) + dzs * muu / (2 * Zs);
    gl += dzp * rho / (2 * Zp);
    gm += dzp * rho / Zp + dzs * rho / (2 * Zs);
    sg[(e * 3 + 0) * NF + fm] = gr;
    sg[(e * 3 + 1) * NF + fm] = gl;
    sg[(e * 3 + 2) * NF + fm] = gm;
  }
  __syncthreads();

  // ---- nodes: one thread per (element, node): the transposed volume term,
  //      the update of the adjoint state, and the volume part of the
  //      gradient.  The gradient's volume terms are sums over nodes of w
  //      times physical derivatives of q; by w^T D q = (D^T w)^T q they are
  //      taken from the transposed derivatives already formed here, dotted
  //      with q at the node, so no forward derivative pass is needed.
  constexpr int UJ = Np % 7 == 0 ? 7 : Np % 5 == 0 ? 5 : 4;  // divides Np
  const int nodes = nE * Np;
  for (int t = tid; t < nodes; t += kT) {
    const int e = t / Np, i = t - e * Np;
    const int64_t k = k0 + e;
    const double *g = smeta + e * DGW_META;
    real X[9];
#pragma unroll
    for (int u = 0; u < 9; ++u) X[u] = (real)g[M_XINV + u];
    const real ri = (real)g[M_RHOINV], la = (real)g[M_LAM], mu = (real)g[M_MU];
    const real *we = sw + e * 9 * Np;
    const real *qe = sq + e * 9 * Np;
    // D_r^T w, D_s^T w, D_t^T w of the nine fields at node i: column i of
    // D_a^T is row i of D_a, stored [j][i] = D(j, i), walked in chunks of
    // immediate offsets
    real ar[9], as[9], at[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) ar[c] = as[c] = at[c] = 0;
    {
      const real *pr = A.Dr + i, *ps = A.Ds + i, *pt = A.Dt + i;
#pragma unroll 1
      for (int j0 = 0; j0 < Np; j0 += UJ) {
        // the chunk's operator entries are loaded together: one round trip
        // per chunk (with this node's lam_q loads after the loop, the
        // registers still allow three waves per SIMD in FP64)
        real a0[UJ], a1[UJ], a2[UJ];
#pragma unroll
        for (int u = 0; u < UJ; ++u) {
          a0[u] = pr[u * Np];
          a1[u] = ps[u * Np];
          a2[u] = pt[u * Np];
        }
#pragma unroll
        for (int u = 0; u < UJ; ++u) {
#pragma unroll
          for (int c = 0; c < 9; ++c) {
            const real x = we[c * Np + j0 + u];
            ar[c] += a0[u] * x;
            as[c] += a1[u] * x;
            at[c] += a2[u] * x;
          }
        }
        pr += UJ * Np;
        ps += UJ * Np;
        pt += UJ * Np;
      }
    }
    // this node's lam_q entries and face positions, loaded together (one by
    // one where they are used, each would cost a full memory round trip:
    // lam_q is written back between them)
    real lqv[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) lqv[c] = lq[(k * 9 + c) * Np + i];
    int mmv[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) mmv[f] = A.facepos[f * Np + i];
    // sum_a X^-1[a][b] (D_a^T w_c) at node i
    auto DTw = [&](int c, int bb) -> real {
      return X[bb] * ar[c] + X[3 + bb] * as[c] + X[6 + bb] * at[c];
    };
    real adj[9];
    // velocity: sum_b d_b^T T_ab, T_aa = la tr(w_s) + 2 mu w_aa, T_ab = mu w_ab
    adj[0] = la * (DTw(3, 0) + DTw(4, 0) + DTw(5, 0)) + 2 * mu * DTw(3, 0) +
             mu * (DTw(8, 1) + DTw(7, 2));
    adj[1] = la * (DTw(3, 1) + DTw(4, 1) + DTw(5, 1)) + 2 * mu * DTw(4, 1) +
             mu * (DTw(8, 0) + DTw(6, 2));
    adj[2] = la * (DTw(3, 2) + DTw(4, 2) + DTw(5, 2)) + 2 * mu * DTw(5, 2) +
             mu * (DTw(7, 0) + DTw(6, 1));
    // stress: (1/rho) d^T of the velocity adjoints
    adj[3] = ri * DTw(0, 0);
    adj[4] = ri * DTw(1, 1);
    adj[5] = ri * DTw(2, 2);
    adj[6] = ri * (DTw(1, 2) + DTw(2, 1));
    adj[7] = ri * (DTw(0, 2) + DTw(2, 0));
    adj[8] = ri * (DTw(0, 1) + DTw(1, 0));
    // volume gradient at node i (FP64 sums), from
    //   rho:    -rho^-2 w_v . div(sigma)
    //   lambda: tr(w_s) div(v)
    //   mu:     2 sum_b w_bb d_b v_b + w_yz (d_z v_y + d_y v_z) + ...
    // with each w . d_b q_c moved onto (D^T w) q_c
    {
      const double q0 = qe[0 * Np + i], q1 = qe[1 * Np + i], q2 = qe[2 * Np + i];
      const double q3 = qe[3 * Np + i], q4 = qe[4 * Np + i], q5 = qe[5 * Np + i];
      const double q6 = qe[6 * Np + i], q7 = qe[7 * Np + i], q8 = qe[8 * Np + i];
      const double rinv = g[M_RHOINV];
      const double sr = (double)DTw(0, 0) * q3 + (double)DTw(0, 1) * q8 +
                        (double)DTw(0, 2) * q7 + (double)DTw(1, 0) * q8 +
                        (double)DTw(1, 1) * q4 + (double)DTw(1, 2) * q6 +
                        (double)DTw(2, 0) * q7 + (double)DTw(2, 1) * q6 +
                        (double)DTw(2, 2) * q5;
      const double sl = (double)(DTw(3, 0) + DTw(4, 0) + DTw(5, 0)) * q0 +
                        (double)(DTw(3, 1) + DTw(4, 1) + DTw(5, 1)) * q1 +
                        (double)(DTw(3, 2) + DTw(4, 2) + DTw(5, 2)) * q2;
      const double sm = 2.0 * ((double)DTw(3, 0) * q0 + (double)DTw(4, 1) * q1 +
                               (double)DTw(5, 2) * q2) +
                        (double)DTw(6, 2) * q1 + (double)DTw(6, 1) * q2 +
                        (double)DTw(7, 2) * q0 + (double)DTw(7, 0) * q2 +
                        (double)DTw(8, 1) * q0 + (double)DTw(8, 0) * q1;
      sgv[(e * 3 + 0) * Np + i] = -rinv * rinv * sr;
      sgv[(e * 3 + 1) * Np + i] = sl;
      sgv[(e * 3 + 2) * Np + i] = sm;
    }
    // the sponge's -sigma q is its own transpose
    if (A.sponge) {
      const real sgm = (real)A.sponge[k];
#pragma unroll
      for (int c = 0; c < 9; ++c) adj[c] -= sgm * we[c * Np + i];
    }
    const real *fa = sfa + e * 9 * NF;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const int mm = mmv[f];
      if (mm >= 0) {
#pragma unroll
        for (int c = 0; c < 9; ++c) adj[c] += fa[c * NF + f * Nfp + mm];
      }
    }
    const real rdt = (real)A.dt, ra = (real)A.rk_a;
    const real nb_ = (real)A.next_b;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      const int64_t idx = (k * 9 + c) * Np + i;
      const real lqn = lqv[c] + rdt * adj[c];
      const real lrn = ra * we[c * Np + i];
      lq[idx] = lqn;
      lr[idx] = lrn;
      // the next stage's w at this node, over this node's own entry of the
      // stage input (read above by this thread only)
      if (A.lift_next) sq[e * 9 * Np + c * Np + i] = lrn + nb_ * lqn;
    }
  }
  __syncthreads();
  // ---- the next reverse stage's lifted adjoint (as adj_lift_kernel) ----
  if (A.lift_next) {
    real *zn_ = A.zbuf_next + (shot * A.K + k0) * 7 * NF;
    for (int t = tid; t < nE * NF; t += kT) {
      const int e = t / NF, fm = t - e * NF, f = fm / Nfp;
      const real *we = sq + e * 9 * Np;
      const double *g = smeta + e * DGW_META;
      real acc[9];
#pragma unroll
      for (int c = 0; c < 9; ++c) acc[c] = 0;
      // fully unrolled: every LIFT entry is loaded before the first is used
#pragma unroll
      for (int i = 0; i < Np; ++i) {
        const real l = A.LIFT[i * NF + fm];
#pragma unroll
        for (int c = 0; c < 9; ++c) acc[c] += l * we[c * Np + i];
      }
      const real fs = (real)g[M_FSCALE + f];
      real z[9];
#pragma unroll
      for (int c = 0; c < 9; ++c) z[c] = fs * acc[c];
      const real ri = (real)g[M_RHOINV];
      const real n0 = (real)g[M_NORMAL + 3 * f], n1 = (real)g[M_NORMAL + 3 * f + 1],
                 n2 = (real)g[M_NORMAL + 3 * f + 2];
      real zc[7];
      zc[0] = ri * z[0];
      zc[1] = ri * z[1];
      zc[2] = ri * z[2];
      zc[3] = 2 * z[3] * n0 + z[8] * n1 + z[7] * n2;
      zc[4] = z[8] * n0 + 2 * z[4] * n1 + z[6] * n2;
      zc[5] = z[7] * n0 + z[6] * n1 + 2 * z[5] * n2;
      zc[6] = z[3] + z[4] + z[5];
#pragma unroll
      for (int c = 0; c < 7; ++c) zn_[(e * 7 + c) * NF + fm] = zc[c];
    }
  }
  // ---- per-element gradient reduction (FP64) --------------------------
  for (int t = tid; t < nE * 3; t += kT) {
    const int e = t / 3, p = t - 3 * e;
    double s = 0.0;
    for (int u = 0; u < NF; ++u) s += sg[(e * 3 + p) * NF + u];
    for (int u = 0; u < Np; ++u) s += sgv[(e * 3 + p) * Np + u];
    A.grad[(shot * A.K + k0 + e) * 3 + p] += A.dt * s;
  }
}

template <typename real>
__global__ void __launch_bounds__(256)
inject_kernel(int Np, real *lam_q, int64_t shot_stride, const int32_t *nrec,
              int rmax, const int32_t *rec_elem, const double *rec_w,
              const double *trace, int64_t cap, const double *d_obs,
              int64_t nobs, const int64_t *shot_step, const int64_t *shot_len,
              double dt) {
  const int shot = blockIdx.y, r = blockIdx.x;
  const int64_t step = shot_step[shot];
  if (step >= shot_len[shot] || step >= cap || step >= nobs) return;
  const int nr = nrec[shot];
  if (r >= nr) return;
  // one work-group per receiver element: the work-group of the element's
  // first receiver adds the contributions of all its receivers, in receiver
  // order (the order of one sequential pass over the receivers), so no two
  // work-groups touch the same entries and each entry is read and written
  // once
  const int32_t *re = rec_elem + (int64_t)shot * rmax;
  const int64_t k = re[r];
  for (int r0 = 0; r0 < r; ++r0)
    if (re[r0] == k) return;   // uniform per work-group
  real *lq = lam_q + shot * shot_stride;
  for (int t = threadIdx.x; t < 3 * Np; t += blockDim.x) {
    const int c = t / Np, j = t - c * Np;
    real v = lq[(k * 9 + c) * Np + j];
    for (int r2 = r; r2 < nr; ++r2) {
      if (re[r2] != k) continue;
      const int64_t base = ((int64_t)shot * rmax + r2) * 3 + c;
      const double res = trace[base * cap + step] - d_obs[base * nobs + step];
      const double add = dt * rec_w[((int64_t)shot * rmax + r2) * Np + j] * res;
      v += (real)add;
    }
    lq[(k * 9 + c) * Np + j] = v;
  }
}

__global__ void set_steps_kernel(int64_t *steps, int n, int64_t value) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) steps[i] = value;
}

template <int N, typename real>
hipError_t adj_launch_t(int nshots, const AdjArgs<real> &a, bool lift, hipStream_t st) {
  constexpr int BE = AdjBlock<N>::be;
  dim3 grid((unsigned)((a.K + BE - 1) / BE), (unsigned)nshots);
  if (lift) {
    hipLaunchKernelGGL((adj_lift_kernel<N, real, BE>), grid, dim3(kT), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((adj_main_kernel<N, real, BE>), grid, dim3(kT), 0, st, a);
  return hipGetLastError();
}

template <typename real>
hipError_t adj_launch_r(int N, int nshots, const void *args, bool lift, hipStream_t st) {
  const AdjArgs<real> &a = *(const AdjArgs<real> *)args;
  switch (N) {
    case 1: return adj_launch_t<1, real>(nshots, a, lift, st);
    case 2: return adj_launch_t<2, real>(nshots, a, lift, st);
    case 3: return adj_launch_t<3, real>(nshots, a, lift, st);
    case 4: return adj_launch_t<4, real>(nshots, a, lift, st);
    case 5: return adj_launch_t<5, real>(nshots, a, lift, st);
    case 6: return adj_launch_t<6, real>(nshots, a, lift, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_adjoint_stage(int N, int precision, int nshots,
                                const void *args, bool lift, hipStream_t st) {
  if (precision == 64) return adj_launch_r<double>(N, nshots, args, lift, st);
  return adj_launch_r<float>(N, nshots, args, lift, st);
}

hipError_t launch_inject(int precision, int nshots, int Np, void *lam_q,
                         int64_t shot_stride, const int32_t *nrec, int rmax,
                         const int32_t *rec_elem, const double *rec_w,
                         const double *trace, int64_t cap, const double *d_obs,
                         int64_t nobs, const int64_t *shot_step,
                         const int64_t *shot_len, double dt, hipStream_t st) {
  if (precision == 64)
    hipLaunchKernelGGL(inject_kernel<double>, dim3(rmax, nshots), dim3(256), 0, st, Np,
                       (double *)lam_q, shot_stride, nrec, rmax, rec_elem, rec_w,
                       trace, cap, d_obs, nobs, shot_step, shot_len, dt);
  else
    hipLaunchKernelGGL(inject_kernel<float>, dim3(rmax, nshots), dim3(256), 0, st, Np,
                       (float *)lam_q, shot_stride, nrec, rmax, rec_elem, rec_w,
                       trace, cap, d_obs, nobs, shot_step, shot_len, dt);
  return hipGetLastError();
}

hipError_t launch_set_steps(int64_t *steps, int nshots, int64_t value,
                            hipStream_t st) {
  hipLaunchKernelGGL(set_steps_kernel, dim3((nshots + 255) / 256), dim3(256), 0,
                     st, steps, nshots, value);
  return hipGetLastError();
}

}  // namespace dgw
