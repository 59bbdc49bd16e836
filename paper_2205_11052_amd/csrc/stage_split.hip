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
// Work item: 16 consecutive elements of one shot (one 16-column MFMA tile per
// component), 6 waves:
//   waves 0-2, velocity component k: rhs_k = sum_a D_a u_{k,a} + LIFT F_k
//     with u_{k,a} = (1/rho) sum_b X^-1[a][b] sigma_kb formed per node from
//     the fields (read from global memory in MFMA lane order) and F_k the
//     lifted velocity flux (LDS): one accumulator per row tile;
//   waves 3-5, velocity component c: D_a v_c for a = 0..2 and the face
//     lifts, accumulated per direction (plus face 0 apart).
// Phases: (1) per-element data to LDS, own and neighbour traces of the
// block's face nodes to registers; (2) exact Riemann flux per face node,
// six quantities to LDS (Fscale dt*/rho and dv); (3) the GEMMs; (4) the
// gradient waves turn their accumulators into G and stage it in LDS over
// the dead flux buffer, while the velocity waves update their component
// straight from the accumulators; (5) all threads form the stress rates
// from G per node and update the six stress components.
#include <hip/hip_runtime.h>

#include <cmath>

#include "dgw_internal.h"
#include "stage_common.h"

namespace dgw {

namespace {

using namespace stagec;

constexpr int kBE = 16;                 // elements per work item (tile width)
constexpr int kWaves = 6;
constexpr int kThr = 64 * kWaves;

template <int N, typename real>
struct SplitSz {
  static constexpr int Np = Sz<N>::Np, Nfp = Sz<N>::Nfp, NF = 4 * Nfp;
  static constexpr int MT = (Np + 15) / 16;   // row tiles of 16 nodes
  static constexpr int KS = (Np + 3) / 4;     // k-steps of one reference derivative
  static constexpr int KL = NF / 4;           // k-steps of the velocity lift
  static constexpr int KF = (Nfp + 3) / 4;    // k-steps of one face's lift
  static constexpr int FLUX = 6 * NF * kBE;   // flux buffer [6][NF][kBE]
  // gradient staging [9][kBE][NpG]: rows of odd length, so the per-lane
  // writes from the accumulators (lanes across elements) spread over the
  // LDS banks and the per-node reads (threads across nodes) are contiguous
  static constexpr int NpG = Np % 2 ? Np : Np + 1;
  static constexpr int GRAD = 9 * kBE * NpG;
  static constexpr int BUF = FLUX > GRAD ? FLUX : GRAD;
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
                KL = Z::KL, KF = Z::KF, FI = Z::FI, NI = Z::NI, NpG = Z::NpG;
  __shared__ double smeta[kBE * DGW_META];
  __shared__ double ssig[kBE];
  __shared__ __attribute__((aligned(16))) real sbuf[Z::BUF];

  const int64_t item = xcd_item(blockIdx.x, total);
  const int shot = (int)(item / nblk);
  const int64_t step = A.shot_step[shot];
  if (step >= A.shot_len[shot]) return;            // uniform per work-group
  const int64_t k0 = (item - (int64_t)shot * nblk) * kBE;
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
      if (j < nE * DGW_META) smeta[j] = mreg[u];
    }
    if (tid < nE) ssig[tid] = A.sponge ? sgv : 0.0;
  }
  // face items t = fm * kBE + e (element fastest, so the flux writes to
  // the [q][fm][kBE] buffer are contiguous across a wave)
  real qm[FI][9], qp[FI][9];
  int cnv[FI];
#pragma unroll
  for (int u = 0; u < FI; ++u) {
    const int t = tid + u * kThr;
    const bool ok = t < kBE * NF && (t & (kBE - 1)) < nE;
    const int tt = ok ? t : 0;
    const int e = tt & (kBE - 1), fm = tt / kBE, f = fm / Nfp;
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
    if (t >= kBE * NF || (t & (kBE - 1)) >= nE) continue;
    const int e = t & (kBE - 1), fm = t / kBE, f = fm / Nfp;
    const double *g = smeta + e * DGW_META;
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
    real *d = sbuf + fm * kBE + e;
    d[0 * NF * kBE] = fs * wx * ri;
    d[1 * NF * kBE] = fs * wy * ri;
    d[2 * NF * kBE] = fs * wz * ri;
    d[3 * NF * kBE] = ux;
    d[4 * NF * kBE] = uy;
    d[5 * NF * kBE] = uz;
  }
  __syncthreads();

  // ---- 3. the GEMMs: one 16-column tile (16 elements, one component) per wave
  const int wave = tid >> 6, lane = tid & 63, g = lane >> 4, col = lane & 15;
  const int ec = col < nE ? col : nE - 1;          // clamped element of this column
  const int64_t kc = k0 + ec;
  const real *qe = qin + kc * 9 * Np;
  const double *gm = smeta + ec * DGW_META;
  const bool velw = wave < 3;
  const int comp = velw ? wave : wave - 3;
  v4 acc[MT], accg[3][MT], acc0[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    acc[mt] = v4{0, 0, 0, 0};
    acc0[mt] = v4{0, 0, 0, 0};
#pragma unroll
    for (int a = 0; a < 3; ++a) accg[a][mt] = v4{0, 0, 0, 0};
  }
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
          acc[mt] = M::mma(Av[((a * KS + ks) * MT + mt) * 64], b, acc[mt]);
      }
    }
    const real *fl = sbuf + comp * NF * kBE + col;
    const real *Al = A.Alift + lane + oz;
#pragma unroll
    for (int ks = 0; ks < KL; ++ks) {
      const real b = fl[(4 * ks + g) * kBE];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
        acc[mt] = M::mma(Al[(ks * MT + mt) * 64], b, acc[mt]);
    }
  } else {
    const real *vc = qe + comp * Np;
    const real *Av = A.Avol + lane + oz;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int j = 4 * ks + g, jj = j < Np ? j : Np - 1;
      real b = vc[jj];
      b = j < Np ? b : (real)0;
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
          accg[a][mt] = M::mma(Av[((a * KS + ks) * MT + mt) * 64], b, accg[a][mt]);
    }
    // face lifts: Alf[f] = c_f LIFT_f (c_0 = 2, c_{1,2,3} = -2), face f > 0
    // into direction f - 1, face 0 apart
    const real *fu = sbuf + (3 + comp) * NF * kBE + col;
    const real *Af = A.Alf + lane + oz;
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
      for (int ks = 0; ks < KF; ++ks) {
        const int m = 4 * ks + g, mm = m < Nfp ? m : Nfp - 1;
        real b = fu[(f * Nfp + mm) * kBE];
        b = m < Nfp ? b : (real)0;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const real a = Af[((f * KF + ks) * MT + mt) * 64];
          if (f == 0)
            acc0[mt] = M::mma(a, b, acc0[mt]);
          else
            accg[f - 1][mt] = M::mma(a, b, accg[f - 1][mt]);
        }
      }
  }
  __syncthreads();   // every wave is done with the flux buffer

  // ---- 4. gradient waves stage G; velocity waves update their component ----
  const real ra = (real)A.rk_a, rb = (real)A.rk_b, rdt = (real)A.dt;
  constexpr bool kStream = N >= 4;
  if (!velw) {
    real X[9];
#pragma unroll
    for (int u = 0; u < 9; ++u) X[u] = (real)gm[M_XINV + u];
    if (col < nE) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * mt + M::row(g, r);
          if (i < Np) {
            const real d0 = accg[0][mt][r] + acc0[mt][r], d1 = accg[1][mt][r] + acc0[mt][r],
                       d2 = accg[2][mt][r] + acc0[mt][r];
#pragma unroll
            for (int b = 0; b < 3; ++b)
              sbuf[((comp * 3 + b) * kBE + col) * NpG + i] =
                  X[b] * d0 + X[3 + b] * d1 + X[6 + b] * d2;
          }
        }
    }
  } else if (col < nE) {
    const real sg = (real)ssig[col];
    const int64_t base = kc * 9 * Np + comp * Np;
    real rold[MT][4], qv[MT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * mt + M::row(g, r), ii = i < Np ? i : Np - 1;
        qv[mt][r] = qin[base + ii];
        if (first)
          rold[mt][r] = (real)0;
        else if constexpr (kStream)
          rold[mt][r] = __builtin_nontemporal_load(res + base + ii);
        else
          rold[mt][r] = res[base + ii];
      }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * mt + M::row(g, r);
        if (i >= Np) continue;
        real rhs = acc[mt][r];
        if (A.sponge) rhs -= sg * qv[mt][r];
        const real rn = first ? rdt * rhs : ra * rold[mt][r] + rdt * rhs;
        const real qn = qv[mt][r] + rb * rn;
        if constexpr (kStream) {
          __builtin_nontemporal_store(rn, res + base + i);
          if constexpr (sizeof(real) == 8)
            __builtin_nontemporal_store(qn, qout + base + i);
          else
            qout[base + i] = qn;
        } else {
          res[base + i] = rn;
          qout[base + i] = qn;
        }
      }
  }
  __syncthreads();

  // ---- 5. stress rates from G per node, source, update of the stresses ----
  const int64_t es = (int64_t)A.src_elem[shot] - k0;   // source element in block
  double s = 0.0;
  const double *spar = A.src_par + 10 * shot;
  if (es >= 0 && es < nE) s = ricker_d(((double)step + A.rk_c) * A.dt, spar[6], spar[7], spar[8]);
#pragma unroll
  for (int u = 0; u < NI; ++u) {
    const int t = tid + u * kThr;
    if (t >= nE * Np) continue;
    const int e = t / Np, i = t - e * Np;
    const double *ge = smeta + e * DGW_META;
    real G[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int b = 0; b < 3; ++b) G[c][b] = sbuf[((c * 3 + b) * kBE + e) * NpG + i];
    const real la = (real)ge[M_LAM], mu = (real)ge[M_MU];
    const real divv = G[0][0] + G[1][1] + G[2][2];
    real rhs[6];
    rhs[0] = la * divv + 2 * mu * G[0][0];
    rhs[1] = la * divv + 2 * mu * G[1][1];
    rhs[2] = la * divv + 2 * mu * G[2][2];
    rhs[3] = mu * (G[1][2] + G[2][1]);
    rhs[4] = mu * (G[0][2] + G[2][0]);
    rhs[5] = mu * (G[0][1] + G[1][0]);
    if (e == es) {
      const double w = s * A.src_vec[shot * Np + i];
#pragma unroll
      for (int c = 0; c < 6; ++c) rhs[c] += (real)(w * spar[c]);
    }
    const int64_t base = (k0 + e) * 9 * Np + 3 * Np + i;
    real qv[6], rold[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      qv[c] = qin[base + c * Np];
      if (first)
        rold[c] = (real)0;
      else if constexpr (kStream)
        rold[c] = __builtin_nontemporal_load(res + base + c * Np);
      else
        rold[c] = res[base + c * Np];
    }
    const real sg = (real)ssig[e];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      real r = rhs[c];
      if (A.sponge) r -= sg * qv[c];
      const real rn = first ? rdt * r : ra * rold[c] + rdt * r;
      const real qn = qv[c] + rb * rn;
      if constexpr (kStream) {
        __builtin_nontemporal_store(rn, res + base + c * Np);
        if constexpr (sizeof(real) == 8)
          __builtin_nontemporal_store(qn, qout + base + c * Np);
        else
          qout[base + c * Np] = qn;
      } else {
        res[base + c * Np] = rn;
        qout[base + c * Np] = qn;
      }
    }
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
