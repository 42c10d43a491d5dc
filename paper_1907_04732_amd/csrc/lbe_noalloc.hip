// lbe_noalloc.hip -- lbe_electrode_charge_noalloc: the electrode charges of
// Gauss's law (Eq. 16 with the Laplacian of Eq. 15) for a potential field in
// caller device memory, computed without allocating anything, for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc).
//
// The per-block partial sums live in `scratch`, a file-scope device array of
// fixed size.  Each GPU holds its own copy of it, at its own address, which
// the host learns once per device with hipGetSymbolAddress; every call on a
// GPU shares that GPU's copy, so calls that overlap on one GPU race.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <mutex>

#include "../../include/lbe.h"
#include "lbe_device.h"
#include "lbe_internal.h"

namespace lbe {
namespace {

constexpr int NA_BLOCK = 256;
constexpr int NA_MAX_BLOCKS = 1024;  // blocks per electrode (grid-stride beyond)
constexpr int NA_MAX_DEVICES = 64;
static_assert(LBE_NOALLOC_MAX_ELECTRODES * NA_MAX_BLOCKS * 2 * 8 <= 512 * 1024,
              "scratch stays modest");

// (sum, compensation) of each block, per electrode: [e][0][b] and [e][1][b].
// Every partial a launch reads is written by the same launch first, so
// nothing needs clearing between calls.
__device__ __align__(256) double scratch[2 * LBE_NOALLOC_MAX_ELECTRODES * NA_MAX_BLOCKS];

// Exact rounding error of t = a + b (Neumaier).
__device__ __forceinline__ double sum_err(double a, double b, double t) {
  return fabs(a) >= fabs(b) ? (a - t) + b : (b - t) + a;
}

// Block tree over (s, c) pairs in a fixed order, carrying each addition's
// exact rounding error into the compensation.
__device__ void block_pair_sum(double &s, double &c, double *ts, double *tc) {
  ts[threadIdx.x] = s;
  tc[threadIdx.x] = c;
  __syncthreads();
  for (int h = NA_BLOCK / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      const double a = ts[threadIdx.x], b = ts[threadIdx.x + h], t = a + b;
      tc[threadIdx.x] += tc[threadIdx.x + h] + sum_err(a, b, t);
      ts[threadIdx.x] = t;
    }
    __syncthreads();
  }
  s = ts[0];
  c = tc[0];
}

// blockIdx.y + 1 = electrode e.  Each thread visits sites r in a grid-stride
// loop; at a solid node of electrode e it forms the node's term of Eq. 16,
// q_scale * sum over links to fluid nodes of wall * w_i (phi(r + c_i) - phi_s(r))
// (links that map the node onto itself, along an axis of size 1, carry
// nothing), and adds it to a compensated running sum.
__global__ __launch_bounds__(NA_BLOCK) void k_charge_scan(Lattice L, double q_scale,
                                                          const uint8_t *__restrict__ type,
                                                          const double *__restrict__ phi,
                                                          double *__restrict__ part) {
  __shared__ double ts[NA_BLOCK], tc[NA_BLOCK];
  const int e = blockIdx.y + 1;
  const int nb = gridDim.x;
  double s = 0.0, c = 0.0;
  for (int r = blockIdx.x * NA_BLOCK + threadIdx.x; r < L.n; r += nb * NA_BLOCK) {
    if (type[r] != e) continue;
    Offs o;
    site_offsets(L, r, o);
    const double ps = phi[r];
    double lap = 0.0;
#pragma unroll
    for (int i = 1; i < NQ; ++i) {
      const int rn = nbr(o, r, i);
      if (rn == r || type[rn] != 0) continue;
      lap += WQ[i] * L.wall * (phi[rn] - ps);
    }
    const double v = q_scale * lap;
    const double t = s + v;
    c += sum_err(s, v, t);
    s = t;
  }
  block_pair_sum(s, c, ts, tc);
  if (threadIdx.x == 0) {
    double *pe = part + (size_t)(e - 1) * 2 * nb;
    pe[blockIdx.x] = s;
    pe[nb + blockIdx.x] = c;
  }
}

// One block per electrode: compensated fold of its blocks' (sum,
// compensation) pairs in a fixed order into q[e - 1].
__global__ __launch_bounds__(NA_BLOCK) void k_charge_fold(const double *__restrict__ part, int nb,
                                                          double *__restrict__ q) {
  __shared__ double ts[NA_BLOCK], tc[NA_BLOCK];
  const double *pe = part + (size_t)blockIdx.x * 2 * nb;
  double s = 0.0, c = 0.0;
  for (int k = threadIdx.x; k < nb; k += NA_BLOCK) {
    const double x = pe[k];
    const double t = s + x;
    c += sum_err(s, x, t) + pe[nb + k];
    s = t;
  }
  block_pair_sum(s, c, ts, tc);
  if (threadIdx.x == 0) q[blockIdx.x] = s + c;
}

std::mutex g_scratch_mu;
double *g_scratch_ptr[NA_MAX_DEVICES] = {};

// The device address of this device's copy of `scratch`, looked up once per
// device (the array's name in host code is a host-side stand-in, not a
// device address).
hipError_t scratch_on(int dev, double **out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (double *)p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

bool device_memory_of(const void *p, int dev) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged) && a.device == dev;
}

}  // namespace
}  // namespace lbe

using namespace lbe;

extern "C" int lbe_electrode_charge_noalloc(int32_t nx, int32_t ny, int32_t nz, double lB,
                                            int32_t flags, const uint8_t *type,
                                            const double *phi, double *q, int32_t ne,
                                            void *stream) {
  if (nx < 1 || ny < 1 || nz < 1)
    return report_init_error(LBE_EINVAL, "lattice dimensions must be >= 1");
  if ((int64_t)nx * ny * nz > LBE_MAX_SITES)
    return report_init_error(LBE_EINVAL, "lattice larger than LBE_MAX_SITES");
  if (ne < 1 || ne > LBE_NOALLOC_MAX_ELECTRODES)
    return report_init_error(LBE_EINVAL,
                             "ne must lie in 1..LBE_NOALLOC_MAX_ELECTRODES (16) for the "
                             "allocation-free charge");
  if (!(lB > 0.0) || !isfinite(lB))
    return report_init_error(LBE_EINVAL, "lB must be finite and > 0");
  if (flags & ~LBE_NAIVE_DIRICHLET)
    return report_init_error(LBE_EINVAL, "only LBE_NAIVE_DIRICHLET is accepted in flags");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NA_MAX_DEVICES)
    return report_init_error(LBE_EDEVICE, "no usable current device");
  if (!type || !phi || !q || !device_memory_of(type, dev) || !device_memory_of(phi, dev) ||
      !device_memory_of(q, dev))
    return report_init_error(LBE_EINVAL,
                             "type, phi and q must be device memory of the current device");
  double *part = nullptr;
  hipError_t e = scratch_on(dev, &part);
  if (e != hipSuccess) return report_init_error(LBE_EDEVICE, hipGetErrorString(e));
  const Lattice L = make_lattice(nx, ny, nz, 0u, (flags & LBE_NAIVE_DIRICHLET) ? 1.0 : 2.0, 0);
  const double q_scale = -6.0 / (4.0 * M_PI * lB);
  const int nb = (int)std::min<long>((L.n + NA_BLOCK - 1) / NA_BLOCK, NA_MAX_BLOCKS);
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_charge_scan, dim3(nb, ne), dim3(NA_BLOCK), 0, s, L, q_scale, type, phi,
                     part);
  hipLaunchKernelGGL(k_charge_fold, dim3(ne), dim3(NA_BLOCK), 0, s, (const double *)part, nb, q);
  e = hipGetLastError();
  if (e != hipSuccess) return report_init_error(LBE_EDEVICE, hipGetErrorString(e));
  return LBE_OK;
}
