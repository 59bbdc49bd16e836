// Allocation-free variant of the energy diagnostic, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid it).
//
// dgw_energy reduces the discrete energy of one shot through a buffer of
// per-work-group partial sums that the library allocates on first use.  The
// variant here keeps that buffer in a file-scope device array instead: one
// copy per GPU, alive until the process ends, whose device address is looked
// up once per device with hipGetSymbolAddress (the array's name in host code
// is only a host-side stand-in and is never passed to a kernel).  The energy
// kernel writes one partial per work-group of 256 elements, every slot it
// uses, so nothing needs clearing; a one-work-group kernel then sums them in
// a fixed order into the slot after the last partial, which is copied to the
// caller.  Calls that overlap on one GPU share the array and race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/dgw.h"
#include "dgw_ctx.h"

namespace {

// Partial sums, one per work-group of 256 elements, plus the total.
constexpr int64_t kMaxPartials = 65536;
constexpr int64_t kMaxElements = kMaxPartials * 256;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kMaxPartials + 1];

double *g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

// Device address of this device's copy of `scratch` (the device must be
// current); null and the HIP error on failure.
hipError_t scratch_ptr(int dev, double **out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = (double *)p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

// One work-group: total of n partials in a fixed order (strided per thread,
// then a tree), written to out[0].
__global__ void __launch_bounds__(256) sum_partials(const double *part, int64_t n,
                                                    double *out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

}  // namespace

extern "C" int dgw_energy_noalloc(dgw_ctx *c, int shot, double *E) {
  if (!c || !E) return DGW_EINVAL;
  if (!c->have_mesh || !c->have_mat) return c->fail(DGW_ESTATE, "mesh and material required");
  if (shot < 0 || shot >= c->nshots) return c->fail(DGW_ERANGE, "shot out of range");
  const int64_t K = c->mesh.K;
  if (K > kMaxElements)
    return c->fail(DGW_ERANGE, "dgw_energy_noalloc supports at most " +
                                   std::to_string(kMaxElements) +
                                   " elements (its static scratch holds " +
                                   std::to_string(kMaxPartials) + " partial sums)");
  int prev = 0;
  hipError_t e = hipGetDevice(&prev);
  if (e != hipSuccess) return c->hipfail(e, "hipGetDevice");
  if (prev != c->device && (e = hipSetDevice(c->device)) != hipSuccess)
    return c->hipfail(e, "hipSetDevice");
  double *sc = nullptr;
  e = scratch_ptr(c->device, &sc);
  int rc = DGW_OK;
  if (e != hipSuccess) {
    rc = c->hipfail(e, "hipGetSymbolAddress(scratch)");
  } else {
    const int64_t nb = (K + 255) / 256;
    const size_t n = (size_t)K * 9 * c->R.Np;
    const char *q = (const char *)c->d_q[c->loc[shot]] + shot * n * c->real_size();
    e = dgw::launch_energy(c->precision, q, K, c->R.Np, c->d_meta,
                           c->have_aniso ? c->d_aniso : nullptr, c->d_M, sc, (int)nb,
                           c->stream);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(sum_partials, dim3(1), dim3(256), 0, c->stream, sc, nb,
                         sc + kMaxPartials);
      e = hipGetLastError();
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(E, sc + kMaxPartials, sizeof(double), hipMemcpyDeviceToHost,
                         c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) rc = c->hipfail(e, "energy (no allocation)");
  }
  if (prev != c->device) (void)hipSetDevice(prev);
  return rc;
}
