// HIP kernels for gfx950: receiver sampling, energy and finiteness
// reductions (the fused stage kernel lives in stage.hip).
#include <hip/hip_runtime.h>

#include <cmath>

#include "dgw_internal.h"

namespace dgw {


// Np is a template parameter so that the weight-times-field loop unrolls
// and each thread issues all of its loads before the first is used (with a
// run-time Np the loads went out a few at a time: 17 us per launch on the
// order-4 benchmark workload).  The sum runs over j in order, as before.
template <typename real, int Np>
__global__ void __launch_bounds__(256) receiver_kernel(RecArgs A) {
  const int shot = blockIdx.x;
  const int64_t step = A.shot_step[shot];
  if (step >= A.shot_len[shot]) return;
  const real *q = (const real *)A.q + shot * A.shot_stride;
  const int nr = A.nrec[shot];
  if (step < A.cap) {
    for (int t = threadIdx.x; t < nr * 3; t += blockDim.x) {
      const int r = t / 3, c = t - 3 * r;
      const int64_t k = A.rec_elem[shot * A.rmax + r];
      const double *w = A.rec_w + ((int64_t)shot * A.rmax + r) * Np;
      const real *qk = q + (k * 9 + c) * Np;
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < Np; ++j) s += w[j] * (double)qk[j];
      A.trace[(((int64_t)shot * A.rmax + r) * 3 + c) * A.cap + step] = s;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) A.shot_step[shot] = step + 1;
}

template <typename real>
__global__ void __launch_bounds__(256)
energy_kernel(const real *q, int64_t K, int Np, const double *meta,
              const double *aniso, const double *M, double *partial) {
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
    if (aniso) {
      // anisotropic: sum_ab S_ab s_a^T M s_b with the compliance S = C^-1
      const double *S = aniso + k * DGW_ANI + A_S;
      double pot = 0.0;
      int u = 0;
      for (int a = 0; a < 6; ++a)
        for (int b = a; b < 6; ++b, ++u) {
          double x = 0.0;
          for (int i = 0; i < Np; ++i) {
            double mi = 0.0;
            for (int j = 0; j < Np; ++j) mi += M[i * Np + j] * (double)qk[(3 + b) * Np + j];
            x += (double)qk[(3 + a) * Np + i] * mi;
          }
          pot += (a == b ? 1.0 : 2.0) * S[u] * x;
        }
      acc += 0.5 * g[M_J] * (rho * kin + pot);
      continue;
    }
    // a fluid element (mu = 0) stores only the isotropic part,
    // tr^T M tr / (9 lambda): the mu -> 0 limit for isotropic stress
    const double pot =
        mu > 0.0 ? (quad[3] + quad[4] + quad[5] + 2.0 * (quad[6] + quad[7] + quad[8])) /
                           (2.0 * mu) -
                       la / (2.0 * mu * (3.0 * la + 2.0 * mu)) * trq
                 : trq / (9.0 * la);
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

template <typename real>
hipError_t launch_receivers_t(int nshots, const RecArgs &a, hipStream_t st) {
  switch (a.Np) {
    case 4: hipLaunchKernelGGL((receiver_kernel<real, 4>), dim3(nshots), dim3(256), 0, st, a); break;
    case 10: hipLaunchKernelGGL((receiver_kernel<real, 10>), dim3(nshots), dim3(256), 0, st, a); break;
    case 20: hipLaunchKernelGGL((receiver_kernel<real, 20>), dim3(nshots), dim3(256), 0, st, a); break;
    case 35: hipLaunchKernelGGL((receiver_kernel<real, 35>), dim3(nshots), dim3(256), 0, st, a); break;
    case 56: hipLaunchKernelGGL((receiver_kernel<real, 56>), dim3(nshots), dim3(256), 0, st, a); break;
    case 84: hipLaunchKernelGGL((receiver_kernel<real, 84>), dim3(nshots), dim3(256), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_receivers(int precision, int nshots, const RecArgs &a,
                            hipStream_t st) {
  if (precision == 64) return launch_receivers_t<double>(nshots, a, st);
  return launch_receivers_t<float>(nshots, a, st);
}

hipError_t launch_energy(int precision, const void *q, int64_t K, int Np,
                         const double *meta, const double *aniso, const double *M,
                         double *partial, int nblocks, hipStream_t st) {
  if (precision == 64)
    hipLaunchKernelGGL(energy_kernel<double>, dim3(nblocks), dim3(256), 0, st,
                       (const double *)q, K, Np, meta, aniso, M, partial);
  else
    hipLaunchKernelGGL(energy_kernel<float>, dim3(nblocks), dim3(256), 0, st,
                       (const float *)q, K, Np, meta, aniso, M, partial);
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
