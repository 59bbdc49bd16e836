// Convolutional perfectly matched layer (C-PML): the memory-variable update
// and the layer's terms, launched after each stage kernel over the layer's
// elements only.
//
// Model (Roden and Gedney 2000; Komatitsch and Martin, Geophysics 72, 2007,
// unsplit first-order form with kappa = 1): in the layer every derivative
// d/dx_b gains a memory variable m with m_t = -(d_b + alpha_b) m - d_b du/dx_b
// (d_b, alpha_b >= 0 per node).  For the velocity-stress system the state
// gains, per node, phi_cb (memory of D_cb = d sigma_cb / dx_b) and psi_cb
// (memory of G_cb = d v_c / dx_b), and the right-hand side gains
//   dL_v = (1/rho) sum_b phi_cb,  dL_sigma = lambda tr(Psi) I + mu (Psi + Psi^T).
// D and G are the scheme's own derivatives split by axis: the volume part
// sum_r Xinv[r][b] D_r u, and the face part Fscale n_b LIFT of the flux-state
// change, with the traction change dT extended to the symmetric stress
// change S = dT n^T + n dT^T - (n.dT) n n^T (S n = dT), so that summed over b
// they give back the scheme's right-hand side.
//
// The stage kernel has already written res' = a res + dt (L q + s) and
// q_out = q_in + b res'.  Adding the layer's terms to L q changes these to
// res' + dt dL and q_out + b dt dL, which this kernel applies to the layer's
// elements; it advances the memory variables with the same LSERK stage
// (mres = a mres + dt m_t, m += b mres), all rates at the stage input.
//
// Two threads per (layer element, node), one for each half of the memory
// variables; the element's fields, per-element data and the lifted face
// quantities are staged in LDS.

#include "dgw_internal.h"
#include "stage_common.h"

namespace dgw {

using stagec::Sz;

namespace {

// 512 threads: 7 layer elements per work-group at order 4 (two 512-thread
// work-groups per CU at 110 VGPRs); 0.48 ms per launch on the order-4 FP64
// benchmark layer against 0.52 ms with 256 threads (3 elements)
constexpr int kPmlThreads = 512;

template <int N>
struct PmlSz {
  static constexpr int Np = Sz<N>::Np;
  // layer elements per work-group: two threads per node
  static constexpr int PB = (kPmlThreads / (2 * Np)) < 32 ? (kPmlThreads / (2 * Np)) : 32;
};

template <int N, typename real>
__global__ void __launch_bounds__(kPmlThreads) pml_kernel(PmlArgs<real> A) {
  constexpr int Np = Sz<N>::Np, Nfp = Sz<N>::Nfp, NF = 4 * Nfp;
  constexpr int PB = PmlSz<N>::PB;
  // per-thread counts of the block's field and per-element loads
  constexpr int NQ = (PB * 9 * Np + kPmlThreads - 1) / kPmlThreads;
  constexpr int NM = (PB * DGW_META + kPmlThreads - 1) / kPmlThreads;
  __shared__ real sq[PB * 9 * Np];
  __shared__ real sfl[PB * NF * 6];
  __shared__ double smeta[PB * DGW_META];
  __shared__ int64_t sk[PB];
  const int shot = A.shot_map ? A.shot_map[blockIdx.y] : (int)blockIdx.y;
  if (A.shot_step[shot] >= A.shot_len[shot]) return;   // uniform per work-group
  const int64_t p0 = (int64_t)blockIdx.x * PB;
  if (p0 >= A.nP) return;
  const int nE = (int)((A.nP - p0) < PB ? (A.nP - p0) : PB);
  const real *__restrict__ qin = A.q_in + shot * A.shot_stride;
  real *__restrict__ qout = A.q_out + shot * A.shot_stride;
  real *__restrict__ res = A.res + shot * A.shot_stride;
  real *__restrict__ mem = A.mem + shot * A.mem_stride;
  real *__restrict__ mres = A.mres + shot * A.mem_stride;
  const int tid = threadIdx.x;

  // The global loads of each phase are unconditional (clamped in-bounds
  // indices, results selected afterwards) and issued before any is waited
  // for: a load under a branch, or one whose use follows it at once, makes
  // the wave wait out a full memory round trip per load.
  if (tid < nE) sk[tid] = A.elem[p0 + tid];
  __syncthreads();
  {
    real vq[NQ];
    double vm[NM];
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
      const int t = tid + j * kPmlThreads;
      const int tc = t < nE * 9 * Np ? t : 0;
      const int e = tc / (9 * Np), r = tc - e * 9 * Np;
      vq[j] = qin[sk[e] * 9 * Np + r];
    }
#pragma unroll
    for (int j = 0; j < NM; ++j) {
      const int t = tid + j * kPmlThreads;
      const int tc = t < nE * DGW_META ? t : 0;
      const int e = tc / DGW_META, r = tc - e * DGW_META;
      vm[j] = A.meta[sk[e] * DGW_META + r];
    }
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
      const int t = tid + j * kPmlThreads;
      if (t < nE * 9 * Np) sq[t] = vq[j];
    }
#pragma unroll
    for (int j = 0; j < NM; ++j) {
      const int t = tid + j * kPmlThreads;
      if (t < nE * DGW_META) smeta[t] = vm[j];
    }
  }
  __syncthreads();

  // ---- faces: the flux-state changes, times Fscale ----
  for (int t = tid; t < nE * NF; t += kPmlThreads) {
    const int e = t / NF, fm = t - e * NF, f = fm / Nfp;
    const int64_t k = sk[e];
    const double *g = smeta + e * DGW_META;
    const real *qe = sq + e * 9 * Np;
    const int n1 = A.fmask[fm];
    const int cn = A.conn[k * 4 + f];
    const int nn = A.nbnode[k * NF + fm];
    // the neighbour's trace, read from the element itself on boundary faces
    const int64_t nb = cn >= 0 ? (int64_t)(cn >> 5) : k;
    const int nc = cn >= 0 ? nn : 0;
    real pn[9], qm[9], p[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) pn[c] = qin[(nb * 9 + c) * Np + nc];
#pragma unroll
    for (int c = 0; c < 9; ++c) qm[c] = qe[c * Np + n1];
    // interior: the neighbour's trace; free surface: the mirror state (v, -sigma);
    // absorbing: the zero state
#pragma unroll
    for (int c = 0; c < 9; ++c)
      p[c] = cn >= 0 ? pn[c] : cn == CONN_FREE ? (c < 3 ? qm[c] : -qm[c]) : (real)0;
    const real nx = (real)g[M_NORMAL + 3 * f], ny = (real)g[M_NORMAL + 3 * f + 1],
               nz = (real)g[M_NORMAL + 3 * f + 2];
    const real dvx = p[0] - qm[0], dvy = p[1] - qm[1], dvz = p[2] - qm[2];
    const real dsxx = p[3] - qm[3], dsyy = p[4] - qm[4], dszz = p[5] - qm[5];
    const real dsyz = p[6] - qm[6], dsxz = p[7] - qm[7], dsxy = p[8] - qm[8];
    const real dtx = dsxx * nx + dsxy * ny + dsxz * nz;
    const real dty = dsxy * nx + dsyy * ny + dsyz * nz;
    const real dtz = dsxz * nx + dsyz * ny + dszz * nz;
    const real dvn = dvx * nx + dvy * ny + dvz * nz;
    const real dtn = dtx * nx + dty * ny + dtz * nz;
    const real zp = (real)g[M_ZP], zs = (real)g[M_ZS];
    const real zpn = (real)g[M_ZPNB + f], zsn = (real)g[M_ZSNB + f];
    const real izp = (real)g[M_IZPS + f], izs = (real)g[M_IZSS + f];
    // the exact Riemann states' changes, blended with the central states'
    // (half the jumps) by the upwind weight
    const real kn = (dtn + zpn * dvn) * izp;
    const real kTx = (dtx - dtn * nx + zsn * (dvx - dvn * nx)) * izs;
    const real kTy = (dty - dtn * ny + zsn * (dvy - dvn * ny)) * izs;
    const real kTz = (dtz - dtn * nz + zsn * (dvz - dvn * nz)) * izs;
    const real tu = A.ftau, hc = ((real)1 - tu) * (real)0.5;
    const real fs = (real)g[M_FSCALE + f];
    real *d = sfl + (e * NF + fm) * 6;
    d[0] = fs * (tu * (zp * kn * nx + zs * kTx) + hc * dtx);
    d[1] = fs * (tu * (zp * kn * ny + zs * kTy) + hc * dty);
    d[2] = fs * (tu * (zp * kn * nz + zs * kTz) + hc * dtz);
    d[3] = fs * (tu * (kn * nx + kTx) + hc * dvx);
    d[4] = fs * (tu * (kn * ny + kTy) + hc * dvy);
    d[5] = fs * (tu * (kn * nz + kTz) + hc * dvz);
  }
  __syncthreads();

  // ---- nodes: directional derivatives, layer terms, memory update ----
  // two threads per node: the first nE Np threads take the velocity
  // derivatives G (memory psi, stress terms), the next nE Np the stress
  // derivatives D (memory phi, velocity terms); each half touches its own
  // nine memory variables and its own fields
  if (tid >= 2 * nE * Np) return;
  const bool vel = tid < nE * Np;
  const int u = vel ? tid : tid - nE * Np;
  const int e = u / Np, i = u - e * Np;
  const int64_t pi = p0 + e;
  const int64_t k = sk[e];
  const real *qe = sq + e * 9 * Np;
  const double *g = smeta + e * DGW_META;
  // an opaque zero added to the operator addresses keeps the compiler from
  // hoisting every operator load out of the chunked loops (far beyond the
  // register file)
  int oz;
  asm volatile("v_mov_b32 %0, 0" : "=v"(oz));
  constexpr int UJ = Np % 7 == 0 ? 7 : Np % 5 == 0 ? 5 : 4;   // divides Np
  // reference derivatives of six fields from c0: the velocity role needs
  // the first three (its other three sums are not used), the stress role
  // all six; the same loop for both keeps it free of branches, so each
  // chunk's operator loads are issued together
  const int c0 = vel ? 0 : 3;
  const real *qc = qe + c0 * Np;
  real acc[6][3];
#pragma unroll
  for (int c = 0; c < 6; ++c) acc[c][0] = acc[c][1] = acc[c][2] = (real)0;
  {
    const real *pr = A.DrT + i + oz, *ps = A.DsT + i + oz, *pt = A.DtT + i + oz;
#pragma unroll 1
    for (int j0 = 0; j0 < Np; j0 += UJ) {
      real a0[UJ], a1[UJ], a2[UJ];
#pragma unroll
      for (int w = 0; w < UJ; ++w) {
        a0[w] = pr[w * Np];
        a1[w] = ps[w * Np];
        a2[w] = pt[w * Np];
      }
#pragma unroll
      for (int w = 0; w < UJ; ++w) {
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          const real v = qc[c * Np + j0 + w];
          acc[c][0] += a0[w] * v;
          acc[c][1] += a1[w] * v;
          acc[c][2] += a2[w] * v;
        }
      }
      pr += UJ * Np;
      ps += UJ * Np;
      pt += UJ * Np;
    }
  }
  real X[9];
#pragma unroll
  for (int w = 0; w < 9; ++w) X[w] = (real)g[M_XINV + w];
  // sigma_cb in Voigt order (xx yy zz yz xz xy) as stress index 0..5
  constexpr int vo[3][3] = {{0, 5, 4}, {5, 1, 3}, {4, 3, 2}};
  real Dg[3][3];   // G (velocity role) or D (stress role), [c][b]
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const real s0 = vel ? acc[c][0] : acc[vo[c][b]][0];
      const real s1 = vel ? acc[c][1] : acc[vo[c][b]][1];
      const real s2 = vel ? acc[c][2] : acc[vo[c][b]][2];
      Dg[c][b] = X[b] * s0 + X[3 + b] * s1 + X[6 + b] * s2;
    }
  // face part: the lifted traction change W (stress role) or velocity
  // change U (velocity role) of each face, with the face's normal
  {
    const real *fle = sfl + e * NF * 6 + (vel ? 3 : 0);
    const real *pl = A.LIFTT + i + oz;
#pragma unroll 1
    for (int f = 0; f < 4; ++f) {
      real l[Nfp];
#pragma unroll
      for (int m = 0; m < Nfp; ++m) l[m] = pl[(f * Nfp + m) * Np];
      real W0 = 0, W1 = 0, W2 = 0;
#pragma unroll
      for (int m = 0; m < Nfp; ++m) {
        const real *s3 = fle + (f * Nfp + m) * 6;
        W0 += l[m] * s3[0];
        W1 += l[m] * s3[1];
        W2 += l[m] * s3[2];
      }
      const real n[3] = {(real)g[M_NORMAL + 3 * f], (real)g[M_NORMAL + 3 * f + 1],
                         (real)g[M_NORMAL + 3 * f + 2]};
      const real Wv[3] = {W0, W1, W2};
      // velocity role: n_b U_c; stress role: n is constant on the face, so
      // the lift of n_b S_cb is n_b (W_c n_b + n_c W_b - n_c n_b (n.W))
      const real nW = n[0] * W0 + n[1] * W1 + n[2] * W2;
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int b = 0; b < 3; ++b)
          Dg[c][b] += vel ? n[b] * Wv[c]
                          : n[b] * (Wv[c] * n[b] + n[c] * Wv[b] - n[c] * n[b] * nW);
    }
  }
  // every remaining load at once: the role's nine memory variables (phi for
  // the stress role, psi for the velocity role) and their residuals, the
  // node's profile, and the residual and output entries the role updates
  // (stress components for the velocity role, velocity for the stress
  // role; the stress role's last three slots repeat its first)
  const int64_t mb = pi * 18 * Np + (vel ? 9 * Np : 0) + i;
  const int nout = vel ? 6 : 3, fb = vel ? 3 : 0;
  real mv[9], mr[9], db[3], ab[3], rv[6], ov[6];
#pragma unroll
  for (int w = 0; w < 9; ++w) mv[w] = mem[mb + w * Np];
#pragma unroll
  for (int w = 0; w < 9; ++w) mr[w] = mres[mb + w * Np];
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    db[b] = (real)A.prof[(pi * 6 + b) * Np + i];
    ab[b] = (real)A.prof[(pi * 6 + 3 + b) * Np + i];
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const int64_t idx = (k * 9 + fb + (c < nout ? c : 0)) * Np + i;
    rv[c] = res[idx];
    ov[c] = qout[idx];
  }
  const real ra = (real)A.rk_a, rb = (real)A.rk_b, rdt = (real)A.dt;
  // the layer's terms: lambda tr(Psi) I + mu (Psi + Psi^T) on sigma
  // (velocity role), or (1/rho) sum_b phi_cb on v_c (stress role)
  real dl[6];
  {
    const real la = (real)g[M_LAM], mu = (real)g[M_MU], ri = (real)g[M_RHOINV];
    const real tr = mv[0] + mv[4] + mv[8];
    const real ds[6] = {la * tr + 2 * mu * mv[0], la * tr + 2 * mu * mv[4],
                        la * tr + 2 * mu * mv[8], mu * (mv[5] + mv[7]),
                        mu * (mv[2] + mv[6]), mu * (mv[1] + mv[3])};
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const int cv = c < 3 ? c : 0;
      const real dv = ri * (mv[3 * cv] + mv[3 * cv + 1] + mv[3 * cv + 2]);
      dl[c] = vel ? ds[c] : dv;
    }
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    if (c < nout) {
      const int64_t idx = (k * 9 + fb + c) * Np + i;
      const real add = rdt * dl[c];
      res[idx] = rv[c] + add;
      qout[idx] = ov[c] + rb * add;
    }
  }
  // memory update: m_t = -(d_b + alpha_b) m_cb - d_b (D or G)_cb; stage 1
  // (a = 0) takes no part of mres, so stale values cannot leak in
  const bool first = A.rk_a == 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const int w = 3 * c + b;
      const real rate = -(db[b] + ab[b]) * mv[w] - db[b] * Dg[c][b];
      const real r = first ? rdt * rate : ra * mr[w] + rdt * rate;
      mres[mb + w * Np] = r;
      mem[mb + w * Np] = mv[w] + rb * r;
    }
}

template <int N, typename real>
hipError_t launch_n(const PmlArgs<real> &a, int nshots, hipStream_t st) {
  constexpr int PB = PmlSz<N>::PB;
  const dim3 grid((unsigned)((a.nP + PB - 1) / PB), (unsigned)nshots);
  hipLaunchKernelGGL((pml_kernel<N, real>), grid, dim3(kPmlThreads), 0, st, a);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_t(int N, const PmlArgs<real> &a, int nshots, hipStream_t st) {
  switch (N) {
    case 1: return launch_n<1, real>(a, nshots, st);
    case 2: return launch_n<2, real>(a, nshots, st);
    case 3: return launch_n<3, real>(a, nshots, st);
    case 4: return launch_n<4, real>(a, nshots, st);
    case 5: return launch_n<5, real>(a, nshots, st);
    case 6: return launch_n<6, real>(a, nshots, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_pml(int N, int precision, int nshots, const void *args, hipStream_t st) {
  if (precision == 64)
    return launch_t<double>(N, *(const PmlArgs<double> *)args, nshots, st);
  return launch_t<float>(N, *(const PmlArgs<float> *)args, nshots, st);
}

}  // namespace dgw
