// Fused right-hand side + LSERK stage kernel on the matrix cores, in the
// minimal operation count ("split" form, launch kernel 2).
//
// The volume term needs 18 reference matrix-vector products per element,
// not 27: nine for the stress divergence of the velocity equation and nine
// reference derivatives of the velocity, from which all six stress rates
// follow by per-node arithmetic.  The face term of the stress equation needs
// one lifted velocity jump per face: with Nanson's relation for an affine
// element, Fscale_f n_f = X^-T c_f with the per-face reference vectors
// c_0 = (2, 2, 2), c_{1,2,3} = -2 e_{0,1,2} (Fscale_f = A_f / J and unit
// face masses), so
//   G_cb = sum_a X^-1[a][b] (D_a v_c + sum_f c_{f,a} LIFT_f dv_{f,c})
// is the velocity gradient plus its lifted face jumps, and the stress rate
// is lambda tr(G) I + mu (G + G^T).  Face f = a + 1 feeds only direction a,
// and face 0 feeds every direction equally, so it has an accumulator of its
// own that is added to each direction.
//
// Work item: 32 consecutive elements of one shot in two tile sets of 16 (one
// 16-column MFMA tile per component and set), 12 waves, six per set:
//   waves 0-2, velocity component k: rhs_k = sum_a D_a u_{k,a} + LIFT F_k
//     with u_{k,a} = (1/rho) sum_b X^-1[a][b] sigma_kb formed per node from
//     the fields (read from global memory in MFMA lane order) and F_k the
//     lifted velocity flux (LDS): one accumulator per row tile;
//   waves 3-5, velocity component c: D_a v_c for a = 0..2 and the face
//     lifts, accumulated per direction (plus face 0 apart).
// One 12-wave work-group fills a CU at the kernel's register budget (three
// waves per SIMD); two six-wave work-groups of 16 elements would not be
// co-resident, since each puts two waves on two of the SIMDs.
// Phases: (1) per-element data to LDS, own and neighbour traces of the
// block's face nodes to registers; (2) exact Riemann flux per face node,
// six quantities to LDS (Fscale dt*/rho and dv); (3) the GEMMs; (4) the
// gradient waves turn their accumulators into G and stage it in LDS over
// the dead flux buffer; (5) the stress rates per node from G, then the whole
// right-hand side (stresses, and the velocity waves' accumulators) to LDS
// in the block's element-field-node order; (6) the point source, sponge and
// LSERK update over the block's contiguous span with 16-byte accesses.
#include <hip/hip_runtime.h>

#include <cmath>

#include "dgw_internal.h"
#include "stage_common.h"

namespace dgw {

namespace {

using namespace stagec;

constexpr int kTile = 16;               // elements per MFMA column tile
constexpr int kSets = 2;                // tile sets per work-group
constexpr int kBE = kTile * kSets;      // elements per work item
constexpr int kWaves = 6 * kSets;       // six waves per tile set
constexpr int kThr = 64 * kWaves;

template <int N, typename real>
struct SplitSz {
  static constexpr int Np = Sz<N>::Np, Nfp = Sz<N>::Nfp, NF = 4 * Nfp;
  static constexpr int MT = (Np + 15) / 16;   // row tiles of 16 nodes
  static constexpr int KS = (Np + 3) / 4;     // k-steps of one reference derivative
  static constexpr int KL = NF / 4;           // k-steps of the velocity lift
  static constexpr int KF = (Nfp + 3) / 4;    // k-steps of one face's lift
  // LDS rows of odd length (in reals or doubles), so lanes that walk across
  // the block's elements at a fixed offset fall in distinct banks
  static constexpr int MS = DGW_META + 1;     // per-element data row
  static constexpr int NFp = NF | 1;          // flux rows [6][kBE][NFp]
  static constexpr int NpG = Np | 1;          // gradient rows [9][kBE][NpG]
  static constexpr int FLUX = 6 * kBE * NFp;
  static constexpr int GRAD = 9 * kBE * NpG;
  static constexpr int RHS = kBE * 9 * Np;    // right-hand side, the block's order
  static constexpr int B1 = FLUX > GRAD ? FLUX : GRAD;
  static constexpr int BUF = B1 > RHS ? B1 : RHS;
  static constexpr int FI = (kBE * NF + kThr - 1) / kThr;   // face items per thread
  static constexpr int NI = (kBE * Np + kThr - 1) / kThr;   // node items per thread
};

// Voigt index of stress component sigma_kb (xx yy zz yz xz xy -> fields 3..8).
__device__ constexpr int sfield(int k, int b) {
  return k == b ? 3 + k : (k + b == 1 ? 8 : (k + b == 2 ? 7 : 6));
}

template <int N, typename real>
__global__ void __launch_bounds__(kThr)
stage_split_kernel(StageArgs<real> A, int64_t nblk, int64_t total) {
  using Z = SplitSz<N, real>;
  using M = Mma<real>;
  using v4 = typename M::v4;
  constexpr int Np = Z::Np, Nfp = Z::Nfp, NF = Z::NF, MT = Z::MT, KS = Z::KS,
                KL = Z::KL, KF = Z::KF, FI = Z::FI, NI = Z::NI, MS = Z::MS,
                NFp = Z::NFp, NpG = Z::NpG;
  __shared__ double smeta[kBE * MS];
  __shared__ double ssig[kBE];
  __shared__ __attribute__((aligned(16))) real sbuf[Z::BUF];
  __shared__ real sf0[3 * kBE * NpG];   // face-0 lift of each velocity component

  const int64_t item = xcd_item(blockIdx.x, total);
  const int slot = (int)(item / nblk);
  const int shot = A.shot_map ? A.shot_map[slot] : slot;
  const int64_t step = A.shot_step[shot];
  if (step >= A.shot_len[shot]) return;            // uniform per work-group
  const int64_t k0 = (item - (int64_t)slot * nblk) * kBE;
  if (k0 >= A.K) return;                           // never taken; bounds nE
  const int nE = (int)((A.K - k0) < kBE ? (A.K - k0) : kBE);
  const real *__restrict__ qin = A.q_in + shot * A.shot_stride;
  real *__restrict__ qout = A.q_out + shot * A.shot_stride;
  real *__restrict__ res = A.res + shot * A.shot_stride;
  const int tid = threadIdx.x;
  const bool first = A.rk_a == 0.0;
  int oz;   // opaque zero for the operator addresses (no hoisting)
  asm volatile("v_mov_b32 %0, 0" : "=v"(oz));

  // ---- 1. per-element data to LDS; traces of the face nodes to registers.
  // Every load is unconditional, out-of-range items reading a clamped
  // in-bounds index whose value is never used.
  {
    const double *mv = A.meta + k0 * DGW_META;
    constexpr int MU = (kBE * DGW_META + kThr - 1) / kThr;
    double mreg[MU];
#pragma unroll
    for (int u = 0; u < MU; ++u) {
      const int j = tid + u * kThr;
      mreg[u] = mv[j < nE * DGW_META ? j : 0];
    }
    const double *sgp = A.sponge ? A.sponge : A.meta;
    const double sgv = sgp[k0 + (tid < nE ? tid : 0)];
#pragma unroll
    for (int u = 0; u < MU; ++u) {
      const int j = tid + u * kThr;
      if (j < nE * DGW_META) smeta[(j / DGW_META) * MS + j % DGW_META] = mreg[u];
    }
    if (tid < nE) ssig[tid] = A.sponge ? sgv : 0.0;
  }
  // face items t = e * NF + fm (face node fastest: a wave's gathers stay
  // within one or two elements)
  real qm[FI][9], qp[FI][9];
  int cnv[FI];
#pragma unroll
  for (int u = 0; u < FI; ++u) {
    const int t = tid + u * kThr;
    const bool ok = t < nE * NF;
    const int tt = ok ? t : 0;
    const int e = tt / NF, fm = tt - e * NF, f = fm / Nfp;
    const int64_t k = k0 + e;
    const int cn = A.conn[k * 4 + f];
    const int nb = A.nbnode[k * NF + fm];
    const int n1 = A.fmask[fm];
    cnv[u] = ok ? cn : CONN_ABSORB;
    const int64_t live = -(int64_t)(ok && cn >= 0);
    const int64_t gb = ((int64_t)(cn >> 5) * 9 * Np + nb) & live;
    const int64_t ob = k * 9 * Np + n1;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      qm[u][c] = qin[ob + c * Np];
      qp[u][c] = qin[gb + c * Np];
    }
  }
  __syncthreads();

  // ---- 2. faces: exact Riemann flux; Fscale dt*/rho and dv to LDS ----
#pragma unroll
  for (int u = 0; u < FI; ++u) {
    const int t = tid + u * kThr;
    if (t >= nE * NF) continue;
    const int e = t / NF, fm = t - e * NF, f = fm / Nfp;
    const double *g = smeta + e * MS;
    real p[9];
    const int cn = cnv[u];
    if (cn >= 0) {
#pragma unroll
      for (int c = 0; c < 9; ++c) p[c] = qp[u][c];
    } else if (cn == CONN_FREE) {
#pragma unroll
      for (int c = 0; c < 3; ++c) p[c] = qm[u][c];
#pragma unroll
      for (int c = 3; c < 9; ++c) p[c] = -qm[u][c];
    } else {
#pragma unroll
      for (int c = 0; c < 9; ++c) p[c] = (real)0;
    }
    const real *m = qm[u];
    const real nx = (real)g[M_NORMAL + 3 * f], ny = (real)g[M_NORMAL + 3 * f + 1],
               nz = (real)g[M_NORMAL + 3 * f + 2];
    const real dvx = p[0] - m[0], dvy = p[1] - m[1], dvz = p[2] - m[2];
    const real dsxx = p[3] - m[3], dsyy = p[4] - m[4], dszz = p[5] - m[5];
    const real dsyz = p[6] - m[6], dsxz = p[7] - m[7], dsxy = p[8] - m[8];
    const real dtx = dsxx * nx + dsxy * ny + dsxz * nz;
    const real dty = dsxy * nx + dsyy * ny + dsyz * nz;
    const real dtz = dsxz * nx + dsyz * ny + dszz * nz;
    const real ri = (real)g[M_RHOINV], fs = (real)g[M_FSCALE + f];
    const real tu = A.ftau, hc = ((real)1 - tu) * (real)0.5;
    const real dvn = dvx * nx + dvy * ny + dvz * nz;
    const real dtn = dtx * nx + dty * ny + dtz * nz;
    const real zp = (real)g[M_ZP], zs = (real)g[M_ZS];
    const real zpn = (real)g[M_ZPNB + f], zsn = (real)g[M_ZSNB + f];
    const real izp = (real)g[M_IZPS + f], izs = (real)g[M_IZSS + f];
    const real kn = (dtn + zpn * dvn) * izp;
    const real kTx = (dtx - dtn * nx + zsn * (dvx - dvn * nx)) * izs;
    const real kTy = (dty - dtn * ny + zsn * (dvy - dvn * ny)) * izs;
    const real kTz = (dtz - dtn * nz + zsn * (dvz - dvn * nz)) * izs;
    const real wx = tu * (zp * kn * nx + zs * kTx) + hc * dtx;
    const real wy = tu * (zp * kn * ny + zs * kTy) + hc * dty;
    const real wz = tu * (zp * kn * nz + zs * kTz) + hc * dtz;
    const real ux = tu * (kn * nx + kTx) + hc * dvx;
    const real uy = tu * (kn * ny + kTy) + hc * dvy;
    const real uz = tu * (kn * nz + kTz) + hc * dvz;
    real *d = sbuf + e * NFp + fm;
    d[0 * kBE * NFp] = fs * wx * ri;
    d[1 * kBE * NFp] = fs * wy * ri;
    d[2 * kBE * NFp] = fs * wz * ri;
    d[3 * kBE * NFp] = ux;
    d[4 * kBE * NFp] = uy;
    d[5 * kBE * NFp] = uz;
  }
  __syncthreads();

  // ---- 3. the GEMMs: one 16-column tile (16 elements, one component) per
  // wave; waves 6 h .. 6 h + 5 own tile set h (elements 16 h .. 16 h + 15)
  const int wave = tid >> 6, lane = tid & 63, g = lane >> 4;
  const int role = wave % 6, col = (wave / 6) * kTile + (lane & 15);
  const int ec = col < nE ? col : nE - 1;          // clamped element of this column
  const int64_t kc = k0 + ec;
  const real *qe = qin + kc * 9 * Np;
  const double *gm = smeta + ec * MS;
  const bool velw = role < 3;
  const int comp = velw ? role : role - 3;
  // one accumulator array for both roles (a wave runs one role, so sharing
  // the registers keeps the other role's tiles out of each branch):
  // velocity waves use acc[0] (their component's right-hand side) and
  // acc[1] (the face-0 lift of velocity component comp, for the gradient
  // waves); gradient waves use acc[a] for reference direction a
  v4 acc[3][MT];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[a][mt] = v4{0, 0, 0, 0};
  if (velw) {
    // u_{k,a} = (1/rho) sum_b X^-1[a][b] sigma_kb
    const real ri = (real)gm[M_RHOINV];
    real cf[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) cf[a][b] = ri * (real)gm[M_XINV + 3 * a + b];
    const real *s0 = qe + sfield(comp, 0) * Np, *s1 = qe + sfield(comp, 1) * Np,
               *s2 = qe + sfield(comp, 2) * Np;
    const real *Av = A.Avol + lane + oz;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int j = 4 * ks + g, jj = j < Np ? j : Np - 1;
      real x0 = s0[jj], x1 = s1[jj], x2 = s2[jj];
      x0 = j < Np ? x0 : (real)0;
      x1 = j < Np ? x1 : (real)0;
      x2 = j < Np ? x2 : (real)0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const real b = cf[a][0] * x0 + cf[a][1] * x1 + cf[a][2] * x2;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
          acc[0][mt] = M::mma(Av[((a * KS + ks) * MT + mt) * 64], b, acc[0][mt]);
      }
    }
    const real *fl = sbuf + (comp * kBE + col) * NFp;
    const real *Al = A.Alift + lane + oz;
#pragma unroll
    for (int ks = 0; ks < KL; ++ks) {
      const real b = fl[4 * ks + g];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
        acc[0][mt] = M::mma(Al[(ks * MT + mt) * 64], b, acc[0][mt]);
    }
    // face-0 lift of velocity component comp (Alf[0] = 2 LIFT_0): the same
    // term for every reference direction of that component's gradient, so
    // it is computed once here and added in the stress assembly
    const real *fu = sbuf + ((3 + comp) * kBE + col) * NFp;
    const real *Af = A.Alf + lane + oz;
#pragma unroll
    for (int ks = 0; ks < KF; ++ks) {
      const int m = 4 * ks + g, mm = m < Nfp ? m : Nfp - 1;
      real b = fu[mm];
      b = m < Nfp ? b : (real)0;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
        acc[1][mt] = M::mma(Af[(ks * MT + mt) * 64], b, acc[1][mt]);
    }
  } else {
    const real *vc = qe + comp * Np;
    const real *Av = A.Avol + lane + oz;
    // software-pipelined: the operator fragments and field value of k-step
    // ks + 1 are loaded before the nine MFMAs of k-step ks, and the
    // scheduling groups keep that order (without them the scheduler sinks
    // every load onto its MFMA and waits on each)
    real an[3][MT], bn;
    auto fetch = [&](int ks) {
      const int j = 4 * ks + g, jj = j < Np ? j : Np - 1;
      bn = vc[jj];
      bn = j < Np ? bn : (real)0;
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) an[a][mt] = Av[((a * KS + ks) * MT + mt) * 64];
    };
    fetch(0);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      real ac[3][MT];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) ac[a][mt] = an[a][mt];
      const real b = bn;
      if (ks + 1 < KS) fetch(ks + 1);
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[a][mt] = M::mma(ac[a][mt], b, acc[a][mt]);
      if (ks + 1 < KS) __builtin_amdgcn_sched_group_barrier(0x020, 3 * MT + 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 3 * MT, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
    // lifts of faces 1-3: Alf[f] = -2 LIFT_f into direction f - 1 (face 0
    // is lifted by the velocity wave of this component)
    // (software-pipelined like the volume loop: operator fragments three
    // k-steps ahead)
    const real *fu = sbuf + ((3 + comp) * kBE + col) * NFp;
    const real *Af = A.Alf + lane + oz;
    constexpr int NIT = 3 * KF, DIST = 3;
    real ring[NIT][MT];
    auto fetchf = [&](int it) {
      const int f = 1 + it / KF, ks = it - (it / KF) * KF;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) ring[it][mt] = Af[((f * KF + ks) * MT + mt) * 64];
    };
#pragma unroll
    for (int it = 0; it < DIST && it < NIT; ++it) fetchf(it);
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int f = 1 + it / KF, ks = it - (it / KF) * KF;
      if (it + DIST < NIT) fetchf(it + DIST);
      const int m = 4 * ks + g, mm = m < Nfp ? m : Nfp - 1;
      real b = fu[f * Nfp + mm];
      b = m < Nfp ? b : (real)0;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[f - 1][mt] = M::mma(ring[it][mt], b, acc[f - 1][mt]);
      if (it + DIST < NIT) __builtin_amdgcn_sched_group_barrier(0x020, MT, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, MT, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  __syncthreads();   // every wave is done with the flux buffer

  // ---- 4. gradient waves: sum_a X^-1[a][b] (D_a v_c + lifts of faces 1-3)
  // to LDS; velocity waves: the face-0 lifts to LDS
  if (velw && col < nE) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * mt + M::row(g, r);
        if (i < Np) sf0[(comp * kBE + col) * NpG + i] = acc[1][mt][r];
      }
  }
  if (!velw && col < nE) {
    real X[9];
#pragma unroll
    for (int u = 0; u < 9; ++u) X[u] = (real)gm[M_XINV + u];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * mt + M::row(g, r);
        if (i < Np) {
          const real d0 = acc[0][mt][r], d1 = acc[1][mt][r], d2 = acc[2][mt][r];
#pragma unroll
          for (int b = 0; b < 3; ++b)
            sbuf[((comp * 3 + b) * kBE + col) * NpG + i] =
                X[b] * d0 + X[3 + b] * d1 + X[6 + b] * d2;
        }
      }
  }
  __syncthreads();

  // ---- 5. stress rates from G per node (to registers); G_cb gains the
  // face-0 lift of v_c times sum_a X^-1[a][b] ----
  real srhs[NI][6];
#pragma unroll
  for (int u = 0; u < NI; ++u) {
    const int t = tid + u * kThr;
    const int tt = t < nE * Np ? t : 0;
    const int e = tt / Np, i = tt - e * Np;
    const double *ge = smeta + e * MS;
    real G[3][3], xs[3];
#pragma unroll
    for (int b = 0; b < 3; ++b)
      xs[b] = (real)ge[M_XINV + b] + (real)ge[M_XINV + 3 + b] + (real)ge[M_XINV + 6 + b];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const real f0 = sf0[(c * kBE + e) * NpG + i];
#pragma unroll
      for (int b = 0; b < 3; ++b) G[c][b] = sbuf[((c * 3 + b) * kBE + e) * NpG + i] + xs[b] * f0;
    }
    const real la = (real)ge[M_LAM], mu = (real)ge[M_MU];
    const real divv = G[0][0] + G[1][1] + G[2][2];
    srhs[u][0] = la * divv + 2 * mu * G[0][0];
    srhs[u][1] = la * divv + 2 * mu * G[1][1];
    srhs[u][2] = la * divv + 2 * mu * G[2][2];
    srhs[u][3] = mu * (G[1][2] + G[2][1]);
    srhs[u][4] = mu * (G[0][2] + G[2][0]);
    srhs[u][5] = mu * (G[0][1] + G[1][0]);
  }
  __syncthreads();   // every G value is read
  // residual loads of this thread's update items (16-byte vectors over the
  // block's contiguous span), issued here -- once the gradient values are
  // consumed, which keeps them clear of the register peak of the stress
  // assembly -- so their latency overlaps the staging below (the state is
  // loaded in the update loop)
  using SP = Span16<real>;
  constexpr int UV = (kBE * 9 * Np / SP::VW + kThr - 1) / kThr;
  constexpr bool kStream = N >= 4;
  const SP sp(shot * A.shot_stride + k0 * 9 * Np, nE * 9 * Np);
  real *rs = res + k0 * 9 * Np, *qo = qout + k0 * 9 * Np;
  const real *qb = qin + k0 * 9 * Np;
  typename SP::vec rv[UV];
#pragma unroll
  for (int u = 0; u < UV; ++u) {
    const int j = tid + u * kThr;
    const int jj = j < sp.nv ? j : (sp.nv > 0 ? sp.nv - 1 : 0);
    const typename SP::vec *rp = (const typename SP::vec *)(rs + sp.hd) + jj;
    if (first)
      rv[u] = typename SP::vec{};
    else if constexpr (kStream)
      rv[u] = __builtin_nontemporal_load(rp);
    else
      rv[u] = *rp;
  }
  const int tl0 = sp.hd + SP::VW * sp.nv;
  const real qh = tid < sp.hd ? qb[tid] : (real)0, qt = tid < sp.tl ? qb[tl0 + tid] : (real)0;
  const real rh = (!first && tid < sp.hd) ? rs[tid] : (real)0;
  const real rt = (!first && tid < sp.tl) ? rs[tl0 + tid] : (real)0;
  // the whole right-hand side to LDS in the block's (element, field, node)
  // order: stresses from the node items, velocities from the accumulators
#pragma unroll
  for (int u = 0; u < NI; ++u) {
    const int t = tid + u * kThr;
    if (t < nE * Np) {
      const int e = t / Np, i = t - e * Np;
#pragma unroll
      for (int c = 0; c < 6; ++c) sbuf[(e * 9 + 3 + c) * Np + i] = srhs[u][c];
    }
  }
  if (velw && col < nE) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * mt + M::row(g, r);
        if (i < Np) sbuf[(col * 9 + comp) * Np + i] = acc[0][mt][r];
      }
  }
  __syncthreads();

  // ---- 6. point source, sponge and LSERK update over the contiguous span
  const real ra = (real)A.rk_a, rb = (real)A.rk_b, rdt = (real)A.dt;
  const int64_t es = (int64_t)A.src_elem[shot] - k0;   // source element in block
  double s = 0.0;
  const double *spar = A.src_par + 10 * shot;
  if (es >= 0 && es < nE) s = ricker_d(((double)step + A.rk_c) * A.dt, spar[6], spar[7], spar[8]);
  auto update = [&](int t, real qold, real rold) -> real2v<real> {
    real rhs = sbuf[t];
    const int e = t / (9 * Np), ci = t - e * 9 * Np, c = ci / Np, i = ci - c * Np;
    if (e == es && c >= 3) rhs += (real)(s * spar[c - 3] * A.src_vec[shot * Np + i]);
    if (A.sponge) rhs -= (real)ssig[e] * qold;
    const real rn = first ? rdt * rhs : ra * rold + rdt * rhs;
    return {rn, qold + rb * rn};
  };
#pragma unroll
  for (int u = 0; u < UV; ++u) {
    const int j = tid + u * kThr;
    if (j >= sp.nv) continue;
    const int b = sp.hd + SP::VW * j;
    const typename SP::vec qv = *(const typename SP::vec *)(qb + b);
    typename SP::vec nr, nq;
#pragma unroll
    for (int l = 0; l < SP::VW; ++l) {
      const real2v<real> o = update(b + l, qv[l], rv[u][l]);
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
    const real2v<real> o = update(tid, qh, rh);
    rs[tid] = o.r;
    qo[tid] = o.q;
  }
  if (tid < sp.tl) {
    const real2v<real> o = update(tl0 + tid, qt, rt);
    rs[tl0 + tid] = o.r;
    qo[tl0 + tid] = o.q;
  }
}

template <int N, typename real>
hipError_t launch_n(int nshots, const StageArgs<real> &a, hipStream_t st) {
  const int64_t nblk = (a.K + kBE - 1) / kBE;
  const int64_t total = nblk * nshots;
  hipLaunchKernelGGL((stage_split_kernel<N, real>), dim3((unsigned)total), dim3(kThr), 0, st,
                     a, nblk, total);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_r(int N, int nshots, const StageArgs<real> &a, hipStream_t st) {
  switch (N) {
    case 1: return launch_n<1, real>(nshots, a, st);
    case 2: return launch_n<2, real>(nshots, a, st);
    case 3: return launch_n<3, real>(nshots, a, st);
    case 4: return launch_n<4, real>(nshots, a, st);
  }
  if constexpr (sizeof(real) == 4) {
    if (N == 5) return launch_n<5, real>(nshots, a, st);
    if (N == 6) return launch_n<6, real>(nshots, a, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace

bool stage_split_supported(int N, int precision) {
  return N >= 1 && (precision == 64 ? N <= 4 : (precision == 32 && N <= 6));
}

int stage_split_block() { return kBE; }

hipError_t launch_stage_split(int N, int precision, int nshots, const void *args,
                              hipStream_t st) {
  if (!stage_split_supported(N, precision)) return hipErrorInvalidValue;
  if (precision == 64) {
    const StageArgs<double> &a = *(const StageArgs<double> *)args;
    if (a.aniso || !a.Avol || !a.Alift || !a.Alf) return hipErrorInvalidValue;
    return launch_r<double>(N, nshots, a, st);
  }
  const StageArgs<float> &a = *(const StageArgs<float> *)args;
  if (a.aniso || !a.Avol || !a.Alift || !a.Alf) return hipErrorInvalidValue;
  return launch_r<float>(N, nshots, a, st);
}

}  // namespace dgw
