// lbe_mg.hip -- geometric multigrid for the Poisson correction equation of
// the LBE step (gfx950).
//
// The outer loop is FP64 defect correction on the paper's equation (Sec. II C):
//   R = L_h phi + 4 pi l_B rho_el  (modified Laplacian of Eq. 15),
//   solve A e = R approximately with A = -L_h,  phi <- phi + e,
// repeated until ||R||_inf <= tol.  The correction e (type T: double in the
// FP64 form, float in the mixed form) is found with one V-cycle.
//
// Levels are cell-centred: a coarse cell is a 2x2x2 block of fine cells
// (a single cell along an axis of size 1, and one half block when a size is
// odd), with block offsets chosen at init so that as few blocks as possible
// mix solid and fluid.  A coarse cell is solid when at least half of its
// children are.  The Dirichlet electrode sits on the face between a fluid and
// a solid cell on every level, so every level uses the same modified stencil
// A e = (6/h^2) sum_i w_i s_i (e - e_i), s_i = 2 towards solid (where e = 0),
// with h = 2^level.  Smoother: four-colour Gauss-Seidel; restriction: mean
// of the fluid children's residuals; prolongation: trilinear between cell
// centres with the value mirrored (-e) across a solid cell, which puts e = 0
// on the wall face.  Coarsest level: one work-group sweeping in LDS-free
// global memory with barriers between colours.
#include <math.h>

#include "lbe_internal.h"

namespace lbe {
namespace {

constexpr int BLOCK = 256;
constexpr int WAVE = 64;
constexpr int COARSE_BLOCK = 1024;

struct Coords {
  int x, y, z;
};

__device__ __forceinline__ Coords coords_of(int r, int nx, int nxy) {
  Coords c;
  c.z = r / nxy;
  const int rem = r - c.z * nxy;
  c.y = rem / nx;
  c.x = rem - c.y * nx;
  return c;
}

__device__ __forceinline__ int wrapi(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

__device__ __forceinline__ int nbr_of(const MgLevel &lv, const Coords &c, int i) {
  return wrapi(c.x + CX[i], lv.nx) + lv.nx * (wrapi(c.y + CY[i], lv.ny) + lv.ny * wrapi(c.z + CZ[i], lv.nz));
}

__device__ __forceinline__ bool solid_link(uint32_t m, int i) { return (m >> (i - 1)) & 1u; }

__device__ __forceinline__ double nanmax(double a, double b) { return (a != a || a > b) ? a : b; }

// A e at a fluid cell, in the level's units: (6/h^2) sum_i w_i s_i (e - e_i)
template <class T>
__device__ __forceinline__ T apply_A(const MgLevel &lv, int r, uint32_t m, const Coords &c,
                                     const T *__restrict__ e) {
  const T er = e[r];
  T acc = T(0);
#pragma unroll
  for (int i = 1; i < NQ; ++i) {
    if ((lv.selfm >> (i - 1)) & 1u) continue;
    const T ws = solid_link(m, i) ? T(2.0 * WQ[i]) : T(WQ[i]);
    acc += ws * (er - e[nbr_of(lv, c, i)]);
  }
  return T(6.0) * T(lv.inv_h2) * acc;
}

// ---- outer residual (FP64) ----------------------------------------------------

template <class T>
__global__ __launch_bounds__(BLOCK) void k_outer_resid(MgLevel lv, const uint32_t *__restrict__ mask,
                                                       const double *__restrict__ src,
                                                       const double *__restrict__ phi,
                                                       T *__restrict__ r0, T *__restrict__ e0,
                                                       double *__restrict__ partial,
                                                       unsigned *__restrict__ counter,
                                                       double *__restrict__ out) {
  __shared__ double sm[BLOCK / WAVE];
  __shared__ double tree[BLOCK];
  __shared__ bool last;
  const int r = blockIdx.x * BLOCK + threadIdx.x;
  double a = 0.0;
  if (r < lv.n) {
    const uint32_t m = mask[r];
    double R = 0.0;
    if (!(m & SOLID_BIT)) {
      const Coords c = coords_of(r, lv.nx, lv.nxy);
      const double ph = phi[r];
      double acc = 0.0;
#pragma unroll
      for (int i = 1; i < NQ; ++i) {
        if ((lv.selfm >> (i - 1)) & 1u) continue;
        const double ws = solid_link(m, i) ? 2.0 * WQ[i] : WQ[i];
        acc += ws * (phi[nbr_of(lv, c, i)] - ph);
      }
      R = 6.0 * (acc + src[r]);
      a = fabs(R);
    }
    r0[r] = T(R);
    e0[r] = T(0);
  }
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) a = nanmax(a, __shfl_xor(a, off));
  if ((threadIdx.x & (WAVE - 1)) == 0) sm[threadIdx.x / WAVE] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < BLOCK / WAVE; ++k) a = nanmax(a, sm[k]);
    partial[blockIdx.x] = a;
    __threadfence();
    last = atomicAdd(counter, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (last) {
    __threadfence();
    double v = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += BLOCK) v = nanmax(v, partial[b]);
    tree[threadIdx.x] = v;
    __syncthreads();
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) tree[threadIdx.x] = nanmax(tree[threadIdx.x], tree[threadIdx.x + s]);
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      out[0] = tree[0];
      atomicExch(counter, 0u);
    }
  }
}

// ---- smoother: one colour of Gauss-Seidel / SOR on A e = r ------------------

template <class T>
__global__ __launch_bounds__(BLOCK) void k_smooth(MgLevel lv, T omega, int colour, int hx, int hy,
                                                  const uint32_t *__restrict__ mask,
                                                  const T *__restrict__ rhs, T *__restrict__ e) {
  const int t = blockIdx.x * BLOCK + threadIdx.x;
  const int plane = hx * hy;
  if (t >= plane * lv.nz) return;
  const int z = t / plane;
  const int rem = t - z * plane;
  const int iy = rem / hx;
  const int ix = rem - iy * hx;
  Coords c;
  c.x = 2 * ix + ((colour ^ z) & 1);
  c.y = 2 * iy + (((colour >> 1) ^ z) & 1);
  c.z = z;
  if (c.x >= lv.nx || c.y >= lv.ny) return;
  const int r = c.x + lv.nx * (c.y + lv.ny * z);
  const uint32_t m = mask[r];
  if (m & SOLID_BIT) return;
  T num = T(0), den = T(0);
#pragma unroll
  for (int i = 1; i < NQ; ++i) {
    if ((lv.selfm >> (i - 1)) & 1u) continue;
    const T ws = solid_link(m, i) ? T(2.0 * WQ[i]) : T(WQ[i]);
    num += ws * e[nbr_of(lv, c, i)];
    den += ws;
  }
  num += T(lv.h2 / 6.0) * rhs[r];
  e[r] = (T(1) - omega) * e[r] + omega * (num / den);
}

// ---- restriction: coarse rhs = mean of the fluid children's residuals -------

template <class T>
__global__ __launch_bounds__(BLOCK) void k_restrict(MgTransfer tr, const uint32_t *__restrict__ mf,
                                                    const uint32_t *__restrict__ mc,
                                                    const T *__restrict__ rf,
                                                    const T *__restrict__ ef, T *__restrict__ rc,
                                                    T *__restrict__ ec) {
  const int R = blockIdx.x * BLOCK + threadIdx.x;
  if (R >= tr.c.n) return;
  ec[R] = T(0);
  if (mc[R] & SOLID_BIT) {
    rc[R] = T(0);
    return;
  }
  const Coords C = coords_of(R, tr.c.nx, tr.c.nxy);
  T sum = T(0);
  int cnt = 0;
  for (int dz = 0; dz < 2; ++dz) {
    const int zp = 2 * C.z + dz;
    if (zp >= tr.f.nz) break;
    const int z = wrapi(zp + tr.oz, tr.f.nz);
    for (int dy = 0; dy < 2; ++dy) {
      const int yp = 2 * C.y + dy;
      if (yp >= tr.f.ny) break;
      const int y = wrapi(yp + tr.oy, tr.f.ny);
      for (int dx = 0; dx < 2; ++dx) {
        const int xp = 2 * C.x + dx;
        if (xp >= tr.f.nx) break;
        const int x = wrapi(xp + tr.ox, tr.f.nx);
        const int r = x + tr.f.nx * (y + tr.f.ny * z);
        const uint32_t m = mf[r];
        if (m & SOLID_BIT) continue;
        Coords c;
        c.x = x;
        c.y = y;
        c.z = z;
        sum += rf[r] - apply_A<T>(tr.f, r, m, c, ef);
        ++cnt;
      }
    }
  }
  rc[R] = cnt ? sum / T(cnt) : T(0);
}

// ---- prolongation: e_f += trilinear interpolation of e_c --------------------

template <class T>
__global__ __launch_bounds__(BLOCK) void k_prolong(MgTransfer tr, const uint32_t *__restrict__ mf,
                                                   const uint32_t *__restrict__ mc,
                                                   const T *__restrict__ ec, T *__restrict__ ef) {
  const int r = blockIdx.x * BLOCK + threadIdx.x;
  if (r >= tr.f.n) return;
  if (mf[r] & SOLID_BIT) return;
  const Coords c = coords_of(r, tr.f.nx, tr.f.nxy);
  // position in the block re-indexing, parent cell and the nearer neighbour
  int P[3], Nb[3];
  const int fx[3] = {wrapi(c.x - tr.ox, tr.f.nx), wrapi(c.y - tr.oy, tr.f.ny), wrapi(c.z - tr.oz, tr.f.nz)};
  const int nf[3] = {tr.f.nx, tr.f.ny, tr.f.nz};
  const int ncs[3] = {tr.c.nx, tr.c.ny, tr.c.nz};
  T wgt[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    P[a] = fx[a] >> 1;
    if (nf[a] == 1) {
      Nb[a] = P[a];
      wgt[a] = T(1);
    } else {
      Nb[a] = wrapi(P[a] + ((fx[a] & 1) ? 1 : -1), ncs[a]);
      wgt[a] = T(0.75);
    }
  }
  const int parent = P[0] + tr.c.nx * (P[1] + tr.c.ny * P[2]);
  const T ep = ec[parent];
  T v = T(0);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int ix = (k & 1) ? Nb[0] : P[0];
    const int iy = (k & 2) ? Nb[1] : P[1];
    const int iz = (k & 4) ? Nb[2] : P[2];
    const T w = ((k & 1) ? T(1) - wgt[0] : wgt[0]) * ((k & 2) ? T(1) - wgt[1] : wgt[1]) *
                ((k & 4) ? T(1) - wgt[2] : wgt[2]);
    if (w == T(0)) continue;
    const int R = ix + tr.c.nx * (iy + tr.c.ny * iz);
    const T val = (mc[R] & SOLID_BIT) ? -ep : ec[R];
    v += w * val;
  }
  if (mc[parent] & SOLID_BIT) v = T(0);
  ef[r] += v;
}

// ---- coarsest level: one work-group, colour sweeps with barriers ------------

template <class T>
__global__ __launch_bounds__(COARSE_BLOCK) void k_coarse(MgLevel lv, T omega, int sweeps,
                                                         const uint32_t *__restrict__ mask,
                                                         const T *__restrict__ rhs,
                                                         T *__restrict__ e) {
  for (int s = 0; s < sweeps; ++s) {
    for (int col = 0; col < 4; ++col) {
      for (int r = threadIdx.x; r < lv.n; r += COARSE_BLOCK) {
        const Coords c = coords_of(r, lv.nx, lv.nxy);
        if ((((c.x + c.z) & 1) + 2 * ((c.y + c.z) & 1)) != col) continue;
        const uint32_t m = mask[r];
        if (m & SOLID_BIT) continue;
        T num = T(0), den = T(0);
#pragma unroll
        for (int i = 1; i < NQ; ++i) {
          if ((lv.selfm >> (i - 1)) & 1u) continue;
          const T ws = solid_link(m, i) ? T(2.0 * WQ[i]) : T(WQ[i]);
          num += ws * e[nbr_of(lv, c, i)];
          den += ws;
        }
        num += T(lv.h2 / 6.0) * rhs[r];
        e[r] = (T(1) - omega) * e[r] + omega * (num / den);
      }
      __threadfence_block();
      __syncthreads();
    }
  }
}

// ---- phi += e --------------------------------------------------------------

template <class T>
__global__ __launch_bounds__(BLOCK) void k_correct(int n, const uint32_t *__restrict__ mask,
                                                   const T *__restrict__ e,
                                                   double *__restrict__ phi) {
  const int r = blockIdx.x * BLOCK + threadIdx.x;
  if (r >= n) return;
  if (mask[r] & SOLID_BIT) return;
  phi[r] += double(e[r]);
}

inline unsigned blocks_for(long n) { return (unsigned)((n + BLOCK - 1) / BLOCK); }

}  // namespace

template <class T>
hipError_t launch_mg_outer_resid(hipStream_t s, const MgLevel &lv, const uint32_t *mask,
                                 const double *src, const double *phi, T *r0, T *e0,
                                 double *partial, unsigned *counter, double *out) {
  hipLaunchKernelGGL(k_outer_resid<T>, dim3(blocks_for(lv.n)), dim3(BLOCK), 0, s, lv, mask, src,
                     phi, r0, e0, partial, counter, out);
  return hipGetLastError();
}

template <class T>
hipError_t launch_mg_smooth(hipStream_t s, const MgLevel &lv, double omega, int colour,
                            const uint32_t *mask, const T *rhs, T *e) {
  const int hx = (lv.nx + 1) / 2, hy = (lv.ny + 1) / 2;
  hipLaunchKernelGGL(k_smooth<T>, dim3(blocks_for((long)hx * hy * lv.nz)), dim3(BLOCK), 0, s, lv,
                     T(omega), colour, hx, hy, mask, rhs, e);
  return hipGetLastError();
}

template <class T>
hipError_t launch_mg_restrict(hipStream_t s, const MgTransfer &tr, const uint32_t *mf,
                              const uint32_t *mc, const T *rf, const T *ef, T *rc, T *ec) {
  hipLaunchKernelGGL(k_restrict<T>, dim3(blocks_for(tr.c.n)), dim3(BLOCK), 0, s, tr, mf, mc, rf,
                     ef, rc, ec);
  return hipGetLastError();
}

template <class T>
hipError_t launch_mg_prolong(hipStream_t s, const MgTransfer &tr, const uint32_t *mf,
                             const uint32_t *mc, const T *ec, T *ef) {
  hipLaunchKernelGGL(k_prolong<T>, dim3(blocks_for(tr.f.n)), dim3(BLOCK), 0, s, tr, mf, mc, ec,
                     ef);
  return hipGetLastError();
}

template <class T>
hipError_t launch_mg_coarse(hipStream_t s, const MgLevel &lv, double omega, int sweeps,
                            const uint32_t *mask, const T *rhs, T *e) {
  hipLaunchKernelGGL(k_coarse<T>, dim3(1), dim3(COARSE_BLOCK), 0, s, lv, T(omega), sweeps, mask,
                     rhs, e);
  return hipGetLastError();
}

template <class T>
hipError_t launch_mg_correct(hipStream_t s, int n, const uint32_t *mask, const T *e,
                             double *phi) {
  hipLaunchKernelGGL(k_correct<T>, dim3(blocks_for(n)), dim3(BLOCK), 0, s, n, mask, e, phi);
  return hipGetLastError();
}

#define LBE_MG_INSTANTIATE(T)                                                                   \
  template hipError_t launch_mg_outer_resid<T>(hipStream_t, const MgLevel &, const uint32_t *,  \
                                               const double *, const double *, T *, T *,       \
                                               double *, unsigned *, double *);                 \
  template hipError_t launch_mg_smooth<T>(hipStream_t, const MgLevel &, double, int,            \
                                          const uint32_t *, const T *, T *);                    \
  template hipError_t launch_mg_restrict<T>(hipStream_t, const MgTransfer &, const uint32_t *,  \
                                            const uint32_t *, const T *, const T *, T *, T *);  \
  template hipError_t launch_mg_prolong<T>(hipStream_t, const MgTransfer &, const uint32_t *,   \
                                           const uint32_t *, const T *, T *);                   \
  template hipError_t launch_mg_coarse<T>(hipStream_t, const MgLevel &, double, int,            \
                                          const uint32_t *, const T *, T *);                    \
  template hipError_t launch_mg_correct<T>(hipStream_t, int, const uint32_t *, const T *,       \
                                           double *);

LBE_MG_INSTANTIATE(double)
LBE_MG_INSTANTIATE(float)

}  // namespace lbe
