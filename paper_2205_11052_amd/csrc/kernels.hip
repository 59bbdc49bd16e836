// HIP kernels for gfx950: fused right-hand side + LSERK stage, receiver
// sampling, energy and finiteness reductions.
//
// Stage kernel (one work-group per block of BE consecutive elements of one
// shot; 256 threads):
//   1. stage the block's fields q[BE][9][Np] (contiguous in HBM, read once,
//      coalesced) and its per-element data into LDS;
//   2. one thread per (element, face node): own trace from LDS, neighbour
//      trace from LDS when the neighbour is in the block, else gathered from
//      HBM/L2 through the face-orientation table; exact Riemann flux written
//      in jump form; the nine lifted flux components (times Fscale) go to LDS;
//   3. one thread per (element, node): reference derivatives of the nine
//      fields with Dr, Ds, Dt, the physical volume terms, + LIFT . flux, +
//      point source, then res = a res + dt rhs and q_out = q_in + b res.
// q_in and q_out are distinct buffers (neighbour traces are read from q_in
// while other blocks write q_out); res is element-local and updated in place.
#include <hip/hip_runtime.h>

#include <cmath>

#include "dgw_internal.h"

namespace dgw {

template <int N>
struct Sz {
  static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  static constexpr int Nfp = (N + 1) * (N + 2) / 2;
};

__device__ inline double ricker_d(double tau, double f0, double t0,
                                  double amp) {
  const double pi = 3.14159265358979323846;
  double a = pi * f0 * (tau - t0);
  a = a * a;
  return amp * (1.0 - 2.0 * a) * exp(-a);
}

constexpr int kThreads = 256;

template <int N, typename real, int BE>
__global__ void __launch_bounds__(kThreads)
stage_kernel(StageArgs<real> A) {
  constexpr int Np = Sz<N>::Np, Nfp = Sz<N>::Nfp, NF = 4 * Nfp;
  __shared__ real sq[BE * 9 * Np];
  __shared__ real sfl[BE * 9 * NF];
  __shared__ double smeta[BE * DGW_META];
  __shared__ int scn[BE * 4];

  const int shot = blockIdx.y;
  const int64_t step = A.shot_step[shot];
  if (step >= A.shot_len[shot]) return;
  const int64_t k0 = (int64_t)blockIdx.x * BE;
  if (k0 >= A.K) return;
  const int nE = (int)((A.K - k0) < BE ? (A.K - k0) : BE);
  const real *__restrict__ qin = A.q_in + shot * A.shot_stride;
  real *__restrict__ qout = A.q_out + shot * A.shot_stride;
  real *__restrict__ res = A.res + shot * A.shot_stride;
  const int tid = threadIdx.x;

  for (int t = tid; t < nE * 9 * Np; t += kThreads) sq[t] = qin[k0 * 9 * Np + t];
  for (int t = tid; t < nE * DGW_META; t += kThreads)
    smeta[t] = A.meta[k0 * DGW_META + t];
  for (int t = tid; t < nE * 4; t += kThreads) scn[t] = A.conn[k0 * 4 + t];
  __syncthreads();

  // ---- faces ----------------------------------------------------------
  for (int t = tid; t < nE * NF; t += kThreads) {
    const int e = t / NF, fm = t - e * NF, f = fm / Nfp, m = fm - f * Nfp;
    const double *g = smeta + e * DGW_META;
    const real *qe = sq + e * 9 * Np;
    const int n1 = A.fmask[fm];
    real qm[9], qp[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) qm[c] = qe[c * Np + n1];
    const int cn = scn[e * 4 + f];
    if (cn >= 0) {
      const int64_t nb = cn >> 5;
      const int f2 = (cn >> 3) & 3, o = cn & 7;
      const int n2 = A.nbtab[((f * 4 + f2) * 6 + o) * Nfp + m];
      const int64_t le = nb - k0;
      if (le >= 0 && le < nE) {
#pragma unroll
        for (int c = 0; c < 9; ++c) qp[c] = sq[le * 9 * Np + c * Np + n2];
      } else {
#pragma unroll
        for (int c = 0; c < 9; ++c) qp[c] = qin[(nb * 9 + c) * Np + n2];
      }
    } else if (cn == CONN_FREE) {
#pragma unroll
      for (int c = 0; c < 3; ++c) qp[c] = qm[c];
#pragma unroll
      for (int c = 3; c < 9; ++c) qp[c] = -qm[c];
    } else {
#pragma unroll
      for (int c = 0; c < 9; ++c) qp[c] = (real)0;
    }
    const real nx = (real)g[M_NORMAL + 3 * f], ny = (real)g[M_NORMAL + 3 * f + 1],
               nz = (real)g[M_NORMAL + 3 * f + 2];
    // jumps [v] = v+ - v-, [t] = (sigma+ - sigma-) n
    const real dvx = qp[0] - qm[0], dvy = qp[1] - qm[1], dvz = qp[2] - qm[2];
    const real dsxx = qp[3] - qm[3], dsyy = qp[4] - qm[4], dszz = qp[5] - qm[5];
    const real dsyz = qp[6] - qm[6], dsxz = qp[7] - qm[7], dsxy = qp[8] - qm[8];
    const real dtx = dsxx * nx + dsxy * ny + dsxz * nz;
    const real dty = dsxy * nx + dsyy * ny + dsyz * nz;
    const real dtz = dsxz * nx + dsyz * ny + dszz * nz;
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
    // dv = v* - v- and dt = t* - t-
    const real Dvx = kn * nx + kTx, Dvy = kn * ny + kTy, Dvz = kn * nz + kTz;
    const real ri = (real)g[M_RHOINV], la = (real)g[M_LAM], mu = (real)g[M_MU];
    const real fs = (real)g[M_FSCALE + f];
    real fl[9];
    fl[0] = (zp * kn * nx + zs * kTx) * ri;
    fl[1] = (zp * kn * ny + zs * kTy) * ri;
    fl[2] = (zp * kn * nz + zs * kTz) * ri;
    const real ndv = nx * Dvx + ny * Dvy + nz * Dvz;
    fl[3] = la * ndv + 2 * mu * Dvx * nx;
    fl[4] = la * ndv + 2 * mu * Dvy * ny;
    fl[5] = la * ndv + 2 * mu * Dvz * nz;
    fl[6] = mu * (Dvy * nz + Dvz * ny);
    fl[7] = mu * (Dvx * nz + Dvz * nx);
    fl[8] = mu * (Dvx * ny + Dvy * nx);
    real *dst = sfl + e * 9 * NF + fm;
#pragma unroll
    for (int c = 0; c < 9; ++c) dst[c * NF] = fs * fl[c];
  }
  __syncthreads();

  // ---- volume + lift + RK update --------------------------------------
  for (int t = tid; t < nE * Np; t += kThreads) {
    const int e = t / Np, i = t - e * Np;
    const real *qe = sq + e * 9 * Np;
    const double *g = smeta + e * DGW_META;
    real dr[9], ds[9], dt[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) dr[c] = ds[c] = dt[c] = (real)0;
    for (int j = 0; j < Np; ++j) {
      const real a0 = A.DrT[j * Np + i], a1 = A.DsT[j * Np + i],
                 a2 = A.DtT[j * Np + i];
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        const real v = qe[c * Np + j];
        dr[c] += a0 * v;
        ds[c] += a1 * v;
        dt[c] += a2 * v;
      }
    }
    real X[9];
#pragma unroll
    for (int u = 0; u < 9; ++u) X[u] = (real)g[M_XINV + u];
    // d/dx_b of field c
    auto D = [&](int c, int b) -> real {
      return X[b] * dr[c] + X[3 + b] * ds[c] + X[6 + b] * dt[c];
    };
    const real ri = (real)g[M_RHOINV], la = (real)g[M_LAM], mu = (real)g[M_MU];
    const real divv = D(0, 0) + D(1, 1) + D(2, 2);
    real rhs[9];
    rhs[0] = (D(3, 0) + D(8, 1) + D(7, 2)) * ri;
    rhs[1] = (D(8, 0) + D(4, 1) + D(6, 2)) * ri;
    rhs[2] = (D(7, 0) + D(6, 1) + D(5, 2)) * ri;
    rhs[3] = la * divv + 2 * mu * D(0, 0);
    rhs[4] = la * divv + 2 * mu * D(1, 1);
    rhs[5] = la * divv + 2 * mu * D(2, 2);
    rhs[6] = mu * (D(1, 2) + D(2, 1));
    rhs[7] = mu * (D(0, 2) + D(2, 0));
    rhs[8] = mu * (D(0, 1) + D(1, 0));
    const real *fle = sfl + e * 9 * NF;
    for (int fm = 0; fm < NF; ++fm) {
      const real l = A.LIFTT[fm * Np + i];
#pragma unroll
      for (int c = 0; c < 9; ++c) rhs[c] += l * fle[c * NF + fm];
    }
    const int64_t k = k0 + e;
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
      const real r = (A.rk_a == 0.0) ? rdt * rhs[c] : ra * res[idx] + rdt * rhs[c];
      res[idx] = r;
      qout[idx] = qe[c * Np + i] + rb * r;
    }
  }
}

template <typename real>
__global__ void __launch_bounds__(256) receiver_kernel(RecArgs A) {
  const int shot = blockIdx.x;
  const int64_t step = A.shot_step[shot];
  if (step >= A.shot_len[shot]) return;
  const real *q = (const real *)A.q + shot * A.shot_stride;
  const int nr = A.nrec[shot];
  const int Np = A.Np;
  if (step < A.cap) {
    for (int t = threadIdx.x; t < nr * 3; t += blockDim.x) {
      const int r = t / 3, c = t - 3 * r;
      const int64_t k = A.rec_elem[shot * A.rmax + r];
      const double *w = A.rec_w + ((int64_t)shot * A.rmax + r) * Np;
      double s = 0.0;
      for (int j = 0; j < Np; ++j) s += w[j] * (double)q[(k * 9 + c) * Np + j];
      A.trace[(((int64_t)shot * A.rmax + r) * 3 + c) * A.cap + step] = s;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) A.shot_step[shot] = step + 1;
}

template <typename real>
__global__ void __launch_bounds__(256)
energy_kernel(const real *q, int64_t K, int Np, const double *meta,
              const double *M, double *partial) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < K;
       k += (int64_t)gridDim.x * blockDim.x) {
    const real *qk = q + k * 9 * Np;
    const double *g = meta + k * DGW_META;
    double quad[9];
    for (int c = 0; c < 9; ++c) quad[c] = 0.0;
    double trq = 0.0;
    for (int i = 0; i < Np; ++i)
      for (int j = 0; j < Np; ++j) {
        const double mij = M[i * Np + j];
        for (int c = 0; c < 9; ++c)
          quad[c] += (double)qk[c * Np + i] * mij * (double)qk[c * Np + j];
        const double ti = (double)qk[3 * Np + i] + (double)qk[4 * Np + i] +
                          (double)qk[5 * Np + i];
        const double tj = (double)qk[3 * Np + j] + (double)qk[4 * Np + j] +
                          (double)qk[5 * Np + j];
        trq += ti * mij * tj;
      }
    const double rho = g[47], la = g[M_LAM], mu = g[M_MU];
    const double kin = quad[0] + quad[1] + quad[2];
    const double pot = (quad[3] + quad[4] + quad[5] +
                        2.0 * (quad[6] + quad[7] + quad[8])) / (2.0 * mu) -
                       la / (2.0 * mu * (3.0 * la + 2.0 * mu)) * trq;
    acc += 0.5 * g[M_J] * (rho * kin + pot);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

template <typename real>
__global__ void __launch_bounds__(256) finite_kernel(const real *q, int64_t n,
                                                     int *flag) {
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite((double)q[i])) bad = 1;
  if (bad) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------
// launch shapes: two elements-per-block choices per order (full and half)

template <int N, typename real>
struct Blocks;
#define DGW_BLOCKS(N_, real_, A_, B_)                 \
  template <>                                         \
  struct Blocks<N_, real_> {                          \
    static constexpr int a = A_, b = B_;              \
  };
DGW_BLOCKS(1, double, 32, 16)
DGW_BLOCKS(2, double, 20, 10)
DGW_BLOCKS(3, double, 12, 6)
DGW_BLOCKS(4, double, 7, 4)
DGW_BLOCKS(5, double, 4, 2)
DGW_BLOCKS(6, double, 3, 2)
DGW_BLOCKS(1, float, 64, 32)
DGW_BLOCKS(2, float, 25, 12)
DGW_BLOCKS(3, float, 12, 6)
DGW_BLOCKS(4, float, 7, 4)
DGW_BLOCKS(5, float, 4, 2)
DGW_BLOCKS(6, float, 3, 2)

template <int N, typename real>
static hipError_t launch_stage_t(int be, int nshots, const StageArgs<real> &a,
                                 hipStream_t st) {
  constexpr int A_ = Blocks<N, real>::a, B_ = Blocks<N, real>::b;
  if (be != A_ && be != B_) return hipErrorInvalidValue;
  const int64_t nb = (a.K + be - 1) / be;
  dim3 grid((unsigned)nb, (unsigned)nshots);
  if (be == A_)
    hipLaunchKernelGGL((stage_kernel<N, real, A_>), grid, dim3(kThreads), 0, st, a);
  else
    hipLaunchKernelGGL((stage_kernel<N, real, B_>), grid, dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

template <typename real>
static hipError_t launch_stage_r(int N, int be, int nshots, const void *args,
                                 hipStream_t st) {
  const StageArgs<real> &a = *(const StageArgs<real> *)args;
  switch (N) {
    case 1: return launch_stage_t<1, real>(be, nshots, a, st);
    case 2: return launch_stage_t<2, real>(be, nshots, a, st);
    case 3: return launch_stage_t<3, real>(be, nshots, a, st);
    case 4: return launch_stage_t<4, real>(be, nshots, a, st);
    case 5: return launch_stage_t<5, real>(be, nshots, a, st);
    case 6: return launch_stage_t<6, real>(be, nshots, a, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_stage(int N, int precision, int be, int nshots,
                        const void *args, hipStream_t st) {
  if (precision == 64) return launch_stage_r<double>(N, be, nshots, args, st);
  return launch_stage_r<float>(N, be, nshots, args, st);
}

template <typename real>
static std::vector<int> choices_r(int N) {
  switch (N) {
    case 1: return {Blocks<1, real>::a, Blocks<1, real>::b};
    case 2: return {Blocks<2, real>::a, Blocks<2, real>::b};
    case 3: return {Blocks<3, real>::a, Blocks<3, real>::b};
    case 4: return {Blocks<4, real>::a, Blocks<4, real>::b};
    case 5: return {Blocks<5, real>::a, Blocks<5, real>::b};
    case 6: return {Blocks<6, real>::a, Blocks<6, real>::b};
  }
  return {};
}

std::vector<int> stage_block_choices(int N, int precision) {
  return precision == 64 ? choices_r<double>(N) : choices_r<float>(N);
}

int default_block(int N, int precision) {
  std::vector<int> c = stage_block_choices(N, precision);
  return c.empty() ? 0 : c[0];
}

hipError_t launch_receivers(int precision, int nshots, const RecArgs &a,
                            hipStream_t st) {
  if (precision == 64)
    hipLaunchKernelGGL(receiver_kernel<double>, dim3(nshots), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(receiver_kernel<float>, dim3(nshots), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_energy(int precision, const void *q, int64_t K, int Np,
                         const double *meta, const double *M, double *partial,
                         int nblocks, hipStream_t st) {
  if (precision == 64)
    hipLaunchKernelGGL(energy_kernel<double>, dim3(nblocks), dim3(256), 0, st,
                       (const double *)q, K, Np, meta, M, partial);
  else
    hipLaunchKernelGGL(energy_kernel<float>, dim3(nblocks), dim3(256), 0, st,
                       (const float *)q, K, Np, meta, M, partial);
  return hipGetLastError();
}

hipError_t launch_finite(int precision, const void *q, int64_t n, int *flag,
                         hipStream_t st) {
  int nb = (int)((n + 255) / 256);
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  if (precision == 64)
    hipLaunchKernelGGL(finite_kernel<double>, dim3(nb), dim3(256), 0, st,
                       (const double *)q, n, flag);
  else
    hipLaunchKernelGGL(finite_kernel<float>, dim3(nb), dim3(256), 0, st,
                       (const float *)q, n, flag);
  return hipGetLastError();
}

}  // namespace dgw
