// lbe_device.h -- device helpers shared by the LBE kernel files (gfx950).
#pragma once

#include <math.h>

#include "lbe_internal.h"

namespace lbe {
namespace {

constexpr int BLOCK = 256;
constexpr int WAVE = 64;

// Periodic neighbour offsets of a site, indexed by c + 1.
struct Offs {
  int x[3], y[3], z[3];
};

__device__ __forceinline__ void site_offsets(const Lattice &L, int r, Offs &o) {
  const int z = r / L.nxy;
  const int rem = r - z * L.nxy;
  const int y = rem / L.nx;
  const int x = rem - y * L.nx;
  o.x[0] = x > 0 ? -1 : L.nx - 1;
  o.x[1] = 0;
  o.x[2] = x + 1 < L.nx ? 1 : 1 - L.nx;
  o.y[0] = y > 0 ? -L.nx : (L.ny - 1) * L.nx;
  o.y[1] = 0;
  o.y[2] = y + 1 < L.ny ? L.nx : -(L.ny - 1) * L.nx;
  o.z[0] = z > 0 ? -L.nxy : (L.nz - 1) * L.nxy;
  o.z[1] = 0;
  o.z[2] = z + 1 < L.nz ? L.nxy : -(L.nz - 1) * L.nxy;
}

__device__ __forceinline__ int nbr(const Offs &o, int r, int i) {
  return r + o.x[CX[i] + 1] + o.y[CY[i] + 1] + o.z[CZ[i] + 1];
}

__device__ __forceinline__ bool solid_link(uint32_t m, int i) { return (m >> (i - 1)) & 1u; }

// Excess (electrostatic) part of the symmetrised link flux of Eq. 10:
//   g = -[n' expm1(delta) - n expm1(-delta)] / (2 Delta),
// with delta = z (phi' - phi - E . c_i); the ideal part is -(n' - n)/Delta.
__device__ __forceinline__ double excess_link(double nh, double nt, double delta, double inv2len) {
  return -(nt * expm1(delta) - nh * expm1(-delta)) * inv2len;
}

// NaN-propagating max
__device__ __forceinline__ double nanmax(double a, double b) { return (a != a || a > b) ? a : b; }

// ---- block reductions -------------------------------------------------------

__device__ double block_max(double v, double *sm) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v = nanmax(v, __shfl_xor(v, off));
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  if (lane == 0) sm[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < BLOCK / WAVE; ++k) v = nanmax(v, sm[k]);
  }
  return v;  // valid in thread 0
}

// pairwise tree sum over the block, fixed order; valid in thread 0
__device__ double block_sum(double v, double *sm) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  __syncthreads();
  if (lane == 0) sm[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) v = (sm[0] + sm[1]) + (sm[2] + sm[3]);
  return v;
}

// True in every thread of the last block to arrive.  The caller's thread 0
// must have written its partial before the call.
__device__ bool arrive_last(unsigned *counter) {
  __shared__ bool last;
  __threadfence();
  if (threadIdx.x == 0) last = atomicAdd(counter, 1u) == gridDim.x - 1;
  __syncthreads();
  if (last) __threadfence();
  return last;
}

inline unsigned blocks_for(long n) { return (unsigned)((n + BLOCK - 1) / BLOCK); }

}  // namespace
}  // namespace lbe
