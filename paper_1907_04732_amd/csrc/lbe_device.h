// lbe_device.h -- device helpers shared by the LBE kernel files (gfx950).
#pragma once

#include <math.h>

#include "lbe_internal.h"

namespace lbe {
namespace {

constexpr int BLOCK = 256;
constexpr int WAVE = 64;

// Logical index of block b of a launch of nb blocks of tb threads over a
// lattice (or level) with nxy sites per z-plane.  The hardware hands out
// blocks round-robin over the NXCD dies (block b to die b mod NXCD), each
// with its own L2, so neighbouring rows and planes, which a stencil reads
// again, would be fetched by several dies.  With `on`, the blocks go in
// chunks of about an eighth of a plane: the j-th block a die receives is
// block j mod chunk of logical chunk (j / chunk) NXCD + die.  The dies then
// sweep the lattice plane by plane, each keeping the same eighth of every
// plane, so a die's next chunk holds the z-neighbours of its last one, and
// the load stays balanced whatever varies along z.  A bijection of [0, nb)
// (blocks past the last whole round of NXCD chunks keep their index), so
// every site is still visited once, and reduction partials stored at the
// logical index keep their order (the results are the same bit for bit).
// Measured on the 192^3 porous electrode it cuts the HBM-side reads of the
// neighbour-gathering kernels by 30-40%, but their time only where it is
// used: the LB pass, the residual checks and the Krylov operator (0.8-2%
// faster) and the FP64 ion pass (same time); the smoothers, the transfers
// and the FP32 ion pass run 1.5-8% slower with it.
__device__ __forceinline__ int xcd_block(int b, int nb, int tb, int nxy, int on) {
  if (!on) return b;
  int chunk = (nxy + tb * NXCD / 2) / (tb * NXCD);
  if (chunk < 1) chunk = 1;
  const int round = NXCD * chunk;
  if (b >= nb - nb % round) return b;
  const int x = b % NXCD, j = b / NXCD;
  return ((j / chunk) * NXCD + x) * chunk + j % chunk;
}

__device__ __forceinline__ int wrapi(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// a / b for 0 <= a < 2^31, 1 <= b, with rb = 1 / b rounded: the product is
// within a/b * 2^-51 of a / b, so its floor is the quotient or one less,
// and one step on the remainder makes it exact (cheaper than an integer
// division by a value known only at run time)
__device__ __forceinline__ int quot(int a, int b, double rb) {
  int q = (int)((double)a * rb);
  if (a - q * b >= b) ++q;
  return q;
}

// Periodic neighbour offsets of a site, indexed by c + 1.
struct Offs {
  int x[3], y[3], z[3];
};

__device__ __forceinline__ void site_offsets(const Lattice &L, int r, Offs &o) {
  const int z = quot(r, L.nxy, L.rnxy);
  const int rem = r - z * L.nxy;
  const int y = quot(rem, L.nx, L.rnx);
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

// A wave-uniform pointer held in scalar registers (readfirstlane of both
// halves), so that the compiler keeps it as the scalar base of ld32/st32
// instead of folding a uniform array offset into per-lane 64-bit addresses.
template <class T>
__device__ __forceinline__ T *sbase(T *p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (T *)(((uint64_t)hi << 32) | lo);
}

// a[i] for an array in global memory (never LDS: the pointer is taken as a
// global one) with a wave-uniform base a (a kernel argument plus a uniform
// array offset such as k N) and a lane's element index i: the byte offset
// stays a 32-bit lane value (i sizeof(T) < 2^32 for i < LBE_MAX_SITES), so
// the access is one scalar-base load or store with no 64-bit address
// arithmetic per lane.
template <class T>
__device__ __forceinline__ T ld32(const T *a, uint32_t i) {
  typedef __attribute__((address_space(1))) const char gchar;
  typedef __attribute__((address_space(1))) const T gT;
  return *(gT *)((gchar *)a + i * (uint32_t)sizeof(T));
}
template <class T>
__device__ __forceinline__ void st32(T *a, uint32_t i, T v) {
  typedef __attribute__((address_space(1))) char gchar;
  typedef __attribute__((address_space(1))) T gT;
  *(gT *)((gchar *)a + i * (uint32_t)sizeof(T)) = v;
}
// ---- LDS plane rings -----------------------------------------------------------
// Where a lattice's (or multigrid level's) nx is a multiple of RING_TX and
// its ny of RING_TY, stencil kernels can take a block of RING_TX x RING_TY
// cells marching along z through a run of zrun planes.
// The planes z - 1, z, z + 1 of the gathered array (with a one-cell halo in
// x and y, wrapped periodically) sit in a ring of four LDS slots, and the
// plane z + 2 travels in registers while the plane z is computed.  Each
// value is then read from memory about once per tile instead of once per
// neighbour: the gathers of the untiled kernels keep the texture units busy
// long before memory is.  A cell sees the same neighbour values as through
// its gathers, so its arithmetic is unchanged.

constexpr int RING_HX = RING_TX + 2, RING_HP = RING_HX * (RING_TY + 2);
constexpr int RING_PER = (RING_HP + BLOCK - 1) / BLOCK;  // halo cells per thread
static_assert(RING_TX * RING_TY == BLOCK, "one cell of a plane per thread");
static_assert(2 * RING_TX == WAVE, "a wavefront holds two rows of a tile");

struct RingTile {
  int x0, y0, z0, zend;  // the tile's corner and its planes [z0, zend), all
                         // before wrapping (an origin offset may push them past
                         // the level's end)
  int lb;                // logical block: reduction partials keep this order
  uint32_t rxy;          // this thread's cell within a plane (wrapped)
  int hc;                // and its halo cell in a slot
};

// Tiles start at the origin (ox, oy, oz): the stencil kernels take 0, the
// restriction its transfer's offsets so that a tile holds whole children
// blocks.
template <class LV>
__device__ __forceinline__ RingTile ring_tile(const LV &lv, int zrun, int ox = 0, int oy = 0,
                                              int oz = 0) {
  const int ntx = lv.nx / RING_TX, nty = lv.ny / RING_TY;
  RingTile t;
  // consecutive tiles of a run of planes on one die, so that the halos they
  // share meet in its L2
  int b = xcd_block(blockIdx.x, gridDim.x, 1, ntx * nty, lv.xcd);
  t.lb = b;
  t.x0 = (b % ntx) * RING_TX + ox;
  b /= ntx;
  t.y0 = (b % nty) * RING_TY + oy;
  t.z0 = (b / nty) * zrun + oz;
  t.zend = min(t.z0 + zrun, lv.nz + oz);
  const int lx = threadIdx.x % RING_TX, ly = threadIdx.x / RING_TX;
  t.rxy = (uint32_t)(wrapi(t.x0 + lx, lv.nx) + lv.nx * wrapi(t.y0 + ly, lv.ny));
  t.hc = (lx + 1) + RING_HX * (ly + 1);
  return t;
}

// This thread's share of a plane's halo cells: loaded into registers by
// fetch, stored into a slot by put.
template <class T>
struct PlaneRing {
  uint32_t gxy[RING_PER];  // offset of the cell within a plane
  int cidx[RING_PER];      // its index in a slot, -1 for none
  T reg[RING_PER];

  template <class LV>
  __device__ __forceinline__ void init(const LV &lv, const RingTile &t) {
#pragma unroll
    for (int j = 0; j < RING_PER; ++j) {
      const int c = threadIdx.x + j * BLOCK;
      cidx[j] = c < RING_HP ? c : -1;
      const int cc = c < RING_HP ? c : 0;
      const int hy = cc / RING_HX, hx = cc - hy * RING_HX;
      const int gx = wrapi(t.x0 + hx - 1, lv.nx), gy = wrapi(t.y0 + hy - 1, lv.ny);
      gxy[j] = (uint32_t)(gx + lv.nx * gy);
    }
  }
  // plane z, wrapped periodically
  template <class LV>
  __device__ __forceinline__ void fetch(const LV &lv, const T *__restrict__ a, int z) {
    const int zz = wrapi(z, lv.nz);
#pragma unroll
    for (int j = 0; j < RING_PER; ++j)
      if (cidx[j] >= 0) reg[j] = ld32(a, gxy[j] + (uint32_t)lv.nxy * (uint32_t)zz);
  }
  __device__ __forceinline__ void put(T *slot) const {
#pragma unroll
    for (int j = 0; j < RING_PER; ++j)
      if (cidx[j] >= 0) slot[cidx[j]] = reg[j];
  }
};

// The slots start as planes z0 - 1 and z0, with z0 + 1 in registers; the
// plane z0 + k then sits in slot (k + 1) & 3.
template <class T, class LV>
__device__ __forceinline__ void ring_start(const LV &lv, const RingTile &t,
                                           PlaneRing<T> &pr, T (*ring)[RING_HP],
                                           const T *__restrict__ a) {
  pr.init(lv, t);
  pr.fetch(lv, a, t.z0 - 1);
  pr.put(ring[0]);
  pr.fetch(lv, a, t.z0);
  pr.put(ring[1]);
  pr.fetch(lv, a, t.z0 + 1);
}

// At plane z: store plane z + 1 into its slot and start loading z + 2.
// The slot written held plane z - 2, read in the previous step, which every
// thread has left at the barrier the caller passes next; so one barrier per
// plane suffices.
template <class T, class LV>
__device__ __forceinline__ void ring_advance(const LV &lv, const RingTile &t, int z,
                                             PlaneRing<T> &pr, T (*ring)[RING_HP],
                                             const T *__restrict__ a) {
  pr.put(ring[(z - t.z0 + 2) & 3]);
  if (z + 1 < t.zend) pr.fetch(lv, a, z + 2);
}

// v[i] = the value at the neighbour c + c_i of this thread's cell in plane z
template <class T>
__device__ __forceinline__ void ring_gather(const RingTile &t, int z, const T (*ring)[RING_HP],
                                            T (&v)[NQ]) {
  const int k = z - t.z0 + 1;
  v[0] = ring[k & 3][t.hc];
#pragma unroll
  for (int i = 1; i < NQ; ++i) v[i] = ring[(k + CZ[i]) & 3][t.hc + CX[i] + RING_HX * CY[i]];
}

// The step passes' streams, each written or read once per pass: with NT as
// non-temporal accesses, which leave the caches to the neighbour data the
// passes re-read.  That pays on lattices whose streams overflow the 256 MB
// last-level cache; on smaller ones the next kernel would find the data
// there, so the context picks NT by the size of its populations.
template <bool NT, class T>
__device__ __forceinline__ void st_stream(T *a, uint32_t i, T v) {
  typedef __attribute__((address_space(1))) char gchar;
  typedef __attribute__((address_space(1))) T gT;
  gT *p = (gT *)((gchar *)a + i * (uint32_t)sizeof(T));
  if (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}
template <bool NT, class T>
__device__ __forceinline__ T ld_stream(const T *p) {
  if (NT) return __builtin_nontemporal_load(p);
  return *p;
}

// v[i] = a[r + c_i] for the 19 velocities (v[0] = a[r]).  Every load is
// unconditional (periodic neighbours are always in range) and issued before
// any value is used, so a wave keeps all of them in flight together instead
// of paying one memory round trip per link behind a branch.
template <class T>
__device__ __forceinline__ void gather(const Offs &o, int r, const T *__restrict__ a, T (&v)[NQ]) {
  v[0] = a[r];
#pragma unroll
  for (int i = 1; i < NQ; ++i) v[i] = a[nbr(o, r, i)];
}

// gather pre-collision populations from the pull-form array (streaming with
// halfway bounce-back): f_i(r) = stored_i(r - c_i), or the node's own
// opposite slot when r - c_i is solid
template <bool NT = false>
__device__ __forceinline__ void pull(const Lattice &L, int r, uint32_t m, const Offs &o,
                                     const double *__restrict__ fin, double (&f)[NQ]) {
  const int N = L.n;
  f[0] = ld_stream<NT>(&fin[r]);
#pragma unroll
  for (int i = 1; i < NQ; ++i) {
    const int j = OPP[i];
    // one unconditional load
    f[i] = ld_stream<NT>(&fin[solid_link(m, j) ? j * N + r : i * N + nbr(o, r, j)]);
  }
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

// ---- second stage of the reductions: one block of FINAL threads combines
// the per-block partials in a fixed order (the kernel boundary orders the
// partial writes before these reads, with no device-wide fence in the first
// stage).  Each thread folds a strided subset with four independent
// accumulators, so the loads of a thread are in flight together.

constexpr int FINAL = 1024;

// sum of partial[0..nb) (fixed order); valid in every thread after the call
__device__ double final_sum(const double *__restrict__ partial, int nb, double *tree) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int b = threadIdx.x;
  for (; b + 3 * FINAL < nb; b += 4 * FINAL) {
    a0 += partial[b];
    a1 += partial[b + FINAL];
    a2 += partial[b + 2 * FINAL];
    a3 += partial[b + 3 * FINAL];
  }
  for (; b < nb; b += FINAL) a0 += partial[b];
  tree[threadIdx.x] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  for (int s = FINAL / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) tree[threadIdx.x] += tree[threadIdx.x + s];
    __syncthreads();
  }
  const double v = tree[0];
  __syncthreads();  // tree may be reused by the caller
  return v;
}

// NaN-propagating max of partial[0..nb) (>= 0 values); valid in every thread.
// The maximum does not depend on the order, so a thread keeps eight loads in
// flight at a time (tens of thousands of partials take few round trips).
__device__ double final_max(const double *__restrict__ partial, int nb, double *tree) {
  constexpr int U = 8;
  double a[U];
#pragma unroll
  for (int j = 0; j < U; ++j) a[j] = 0.0;
  int b = threadIdx.x;
  for (; b + (U - 1) * FINAL < nb; b += U * FINAL) {
    double v[U];
#pragma unroll
    for (int j = 0; j < U; ++j) v[j] = partial[b + j * FINAL];
#pragma unroll
    for (int j = 0; j < U; ++j) a[j] = nanmax(a[j], v[j]);
  }
  for (; b < nb; b += FINAL) a[0] = nanmax(a[0], partial[b]);
#pragma unroll
  for (int j = 1; j < U; ++j) a[0] = nanmax(a[0], a[j]);
  tree[threadIdx.x] = a[0];
  __syncthreads();
  for (int s = FINAL / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) tree[threadIdx.x] = nanmax(tree[threadIdx.x], tree[threadIdx.x + s]);
    __syncthreads();
  }
  const double v = tree[0];
  __syncthreads();
  return v;
}

// out[0] = max over partial[0..nb)
__global__ __launch_bounds__(FINAL) void k_final_max(const double *__restrict__ partial, int nb,
                                                     double *__restrict__ out) {
  __shared__ double tree[FINAL];
  const double v = final_max(partial, nb, tree);
  if (threadIdx.x == 0) out[0] = v;
}

// Residual check of a Poisson solve: max over the block maxima into
// ctl->resid; marks the solve done when the residual is <= tol or not finite.
__global__ __launch_bounds__(FINAL) void k_final_resid(const double *__restrict__ partial, int nb,
                                                       SolveCtl *__restrict__ ctl, int add) {
  __shared__ double tree[FINAL];
  if (ctl->done) return;
  const double res = final_max(partial, nb, tree);
  if (threadIdx.x == 0) {
    const int count = ctl->count + add;
    ctl->count = count;
    ctl->resid = res;
    ctl->checks += 1;
    const bool bad = !(res == res) || res > 1.7976931348623157e308;
    if (bad || (ctl->tol > 0.0 && res <= ctl->tol)) {
      ctl->done = 1;
      ctl->iters = count;
      ctl->nonfinite = bad;
    }
    // publish to the host: the values first, then (after a system-scope
    // fence) the stamp the host polls on, in one 8-byte store, which the end
    // of the kernel makes visible at the latest
    if (ctl->mirror) {
      volatile SolveCtl *hm = ctl->mirror;
      hm->resid = res;
      hm->count = count;
      hm->iters = ctl->iters;
      hm->nonfinite = ctl->nonfinite;
      __threadfence_system();
      hm->stamp = ((unsigned long long)(unsigned)ctl->seq << 32) |
                  ((unsigned long long)(ctl->done ? 1u : 0u) << 31) |
                  (unsigned long long)(unsigned)ctl->checks;
    }
  }
}

// out[q] = sum over partial[q*nb .. q*nb + nb), q < nq (fixed order)
__global__ __launch_bounds__(FINAL) void k_final_sum(const double *__restrict__ partial, int nb,
                                                     int nq, double *__restrict__ out) {
  __shared__ double tree[FINAL];
  for (int q = 0; q < nq; ++q) {
    const double v = final_sum(partial + (size_t)q * nb, nb, tree);
    if (threadIdx.x == 0) out[q] = v;
  }
}

// ---- the link-flux exponentials -------------------------------------------
// The symmetrised flux of Eq. 10 needs n' e^delta - n e^-delta.  Writing
// e^(+-delta) = 1 + C +- S with S = sinh(delta), C = cosh(delta) - 1 gives
//   n' expm1(delta) - n expm1(-delta) = (n' + n) S + (n' - n) C
// exactly.  For |delta| <= 1/2 both come from their Taylor series (next
// terms below 1e-17 relative); beyond, from expm1.

constexpr double TAYLOR_MAX = 0.5;  // |delta| up to which the series are used

__device__ __forceinline__ void sinh_coshm1_series(double d, double &S, double &C) {
  const double x = d * d;
  S = d * (1.0 + x * (1.0 / 6 + x * (1.0 / 120 + x * (1.0 / 5040 + x * (1.0 / 362880 +
           x * (1.0 / 39916800 + x * (1.0 / 6227020800.0)))))));
  C = x * (0.5 + x * (1.0 / 24 + x * (1.0 / 720 + x * (1.0 / 40320 + x * (1.0 / 3628800 +
           x * (1.0 / 479001600 + x * (1.0 / 87178291200.0)))))));
}

__device__ __forceinline__ void sinh_coshm1(double d, double &S, double &C) {
  if (fabs(d) <= TAYLOR_MAX) {
    sinh_coshm1_series(d, S, C);
  } else {
    const double ep = expm1(d), em = expm1(-d);
    S = 0.5 * (ep - em);
    C = 0.5 * (ep + em);
  }
}

// sinh and cosh - 1 of z delta for valence z, from S1, C1 of delta: for
// z = +-1 they are reused (both the series and the expm1 form are exactly odd
// and even in delta, so the values equal a direct evaluation bit for bit);
// other valences are evaluated directly.  z is uniform across the launch.
__device__ __forceinline__ void valence_sc(int z, double delta, double S1, double C1, double &S,
                                           double &C) {
  if (z == 1) {
    S = S1;
    C = C1;
  } else if (z == -1) {
    S = -S1;
    C = C1;
  } else {
    sinh_coshm1(z * delta, S, C);
  }
}

// Excess (electrostatic) part of the symmetrised link flux of Eq. 10:
//   g = -[n' expm1(delta) - n expm1(-delta)] / (2 Delta),
// with delta = z (phi' - phi - E . c_i); the ideal part is -(n' - n)/Delta.
__device__ __forceinline__ double excess_link(double nh, double nt, double delta, double inv2len) {
  double S, C;
  sinh_coshm1(delta, S, C);
  return -((nt + nh) * S + (nt - nh) * C) * inv2len;
}

// the series branch only (valid for |delta| <= TAYLOR_MAX); branch-free
__device__ __forceinline__ double excess_link_series(double nh, double nt, double delta,
                                                     double inv2len) {
  double S, C;
  sinh_coshm1_series(delta, S, C);
  return -((nt + nh) * S + (nt - nh) * C) * inv2len;
}

// Knuth's two-sum: s + e == a + b exactly, s = fl(a + b), for any a, b (no
// ordering of magnitudes needed; six additions, none contracted or
// reassociated at -O3 without fast-math).
__device__ __forceinline__ void two_sum_f(float a, float b, float &s, float &e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void sinh_coshm1f_series(float d, float &S, float &C) {
  const float x = d * d;
  S = d * (1.f + x * (1.f / 6 + x * (1.f / 120 + x * (1.f / 5040 + x * (1.f / 362880)))));
  C = x * (0.5f + x * (1.f / 24 + x * (1.f / 720 + x * (1.f / 40320 + x * (1.f / 3628800)))));
}

__device__ __forceinline__ void sinh_coshm1f(float d, float &S, float &C) {
  if (fabsf(d) <= float(TAYLOR_MAX)) {
    sinh_coshm1f_series(d, S, C);
  } else {
    const float ep = expm1f(d), em = expm1f(-d);
    S = 0.5f * (ep - em);
    C = 0.5f * (ep + em);
  }
}

__device__ __forceinline__ void valence_scf(int z, double delta, float d1, float S1, float C1,
                                            float &S, float &C) {
  if (z == 1) {
    S = S1;
    C = C1;
  } else if (z == -1) {
    S = -S1;
    C = C1;
  } else {
    sinh_coshm1f(float(z * delta), S, C);
  }
  (void)d1;
}

__device__ __forceinline__ float excess_link_f(float nh, float nt, float delta, float inv2len) {
  float S, C;
  sinh_coshm1f(delta, S, C);
  return -((nt + nh) * S + (nt - nh) * C) * inv2len;
}

__device__ __forceinline__ float excess_link_f_series(float nh, float nt, float delta,
                                                      float inv2len) {
  float S, C;
  sinh_coshm1f_series(delta, S, C);
  return -((nt + nh) * S + (nt - nh) * C) * inv2len;
}

// Warm start of the next Poisson solve at fluid node r: phi extrapolated in
// time from the last converged potentials prev = [phi(t-1) | phi(t-2)]
// (order 2: 3 phi - 3 p1 + p2, quadratic; 1: 2 phi - p1; 0: phi), then the
// history shifts.  Run by the ion pass, which does not read phi.  Every node
// runs it so that each store writes whole cache lines: a solid node writes
// its potential (the electrode's) back unchanged and zeros into the history,
// which is never read there and starts at zero.
__device__ __forceinline__ void extrapolate_at(int r, int n, int order, bool solid,
                                               double *__restrict__ phi,
                                               double *__restrict__ prev) {
  const double now = phi[r];
  if (order < 0) {  // no extrapolation: only keep phi(t)
    prev[r] = now;
    return;
  }
  const double p1 = prev[r];
  double next = now;
  if (!solid) {
    if (order >= 2) next = 3.0 * (now - p1) + prev[n + r];
    else if (order == 1) next = 2.0 * now - p1;
  }
  phi[r] = next;
  prev[n + r] = solid ? 0.0 : p1;
  prev[r] = solid ? 0.0 : now;
}

inline unsigned blocks_for(long n) { return (unsigned)((n + BLOCK - 1) / BLOCK); }

// The step passes come in three block sizes (the launch shape the context
// picked by timing them, see lbe_capi.cpp): CALL(KK, TB) for species count K
// and block size TBV (128, 256 or 512; anything else: 256).
#define LBE_DISPATCH_TB(KK, TBV, CALL) \
  switch (TBV) {                       \
    case 128: CALL(KK, 128); break;    \
    case 512: CALL(KK, 512); break;    \
    default: CALL(KK, 256); break;     \
  }
#define LBE_DISPATCH_K_TB(K, TBV, CALL)           \
  switch (K) {                                    \
    case 1: LBE_DISPATCH_TB(1, TBV, CALL) break;  \
    case 2: LBE_DISPATCH_TB(2, TBV, CALL) break;  \
    case 3: LBE_DISPATCH_TB(3, TBV, CALL) break;  \
    default: LBE_DISPATCH_TB(4, TBV, CALL) break; \
  }
// ... and with the stream kind of the step passes: CALL(KK, TB, NT), NT
// true for non-temporal population and output streams
#define LBE_DISPATCH_TB_NT(KK, TBV, NT, CALL) \
  switch (TBV) {                              \
    case 128: CALL(KK, 128, NT); break;       \
    case 512: CALL(KK, 512, NT); break;       \
    default: CALL(KK, 256, NT); break;        \
  }
#define LBE_DISPATCH_K_NT(K, TBV, NT, CALL)               \
  switch (K) {                                            \
    case 1: LBE_DISPATCH_TB_NT(1, TBV, NT, CALL) break;   \
    case 2: LBE_DISPATCH_TB_NT(2, TBV, NT, CALL) break;   \
    case 3: LBE_DISPATCH_TB_NT(3, TBV, NT, CALL) break;   \
    default: LBE_DISPATCH_TB_NT(4, TBV, NT, CALL) break;  \
  }
#define LBE_DISPATCH_K_TB_NT(K, TBV, NTV, CALL) \
  if (NTV) {                                    \
    LBE_DISPATCH_K_NT(K, TBV, true, CALL)       \
  } else {                                      \
    LBE_DISPATCH_K_NT(K, TBV, false, CALL)      \
  }

}  // namespace
}  // namespace lbe
