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

#include "lbe_device.h"
#include "lbe_internal.h"

namespace lbe {
namespace {

constexpr int COARSE_BLOCK = 1024;

struct Coords {
  int x, y, z;
};

__device__ __forceinline__ Coords coords_of(int r, const MgLevel &lv) {
  Coords c;
  c.z = quot(r, lv.nxy, lv.rnxy);
  const int rem = r - c.z * lv.nxy;
  c.y = quot(rem, lv.nx, lv.rnx);
  c.x = rem - c.y * lv.nx;
  return c;
}

__device__ __forceinline__ int nbr_of(const MgLevel &lv, const Coords &c, int i) {
  return wrapi(c.x + CX[i], lv.nx) + lv.nx * (wrapi(c.y + CY[i], lv.ny) + lv.ny * wrapi(c.z + CZ[i], lv.nz));
}

// v[i] = e at the neighbour c + c_i of a level's cell (v[0] = e[r]); all loads
// are issued before any value is used.  The wrapped offsets along each axis
// are formed once per cell, so a neighbour's index is one add per axis.
template <class T>
__device__ __forceinline__ void gather_lv(const MgLevel &lv, const Coords &c, int r,
                                          const T *__restrict__ e, T (&v)[NQ]) {
  const int ox[3] = {c.x > 0 ? -1 : lv.nx - 1, 0, c.x + 1 < lv.nx ? 1 : 1 - lv.nx};
  const int oy[3] = {c.y > 0 ? -lv.nx : (lv.ny - 1) * lv.nx, 0,
                     c.y + 1 < lv.ny ? lv.nx : -(lv.ny - 1) * lv.nx};
  const int oz[3] = {c.z > 0 ? -lv.nxy : (lv.nz - 1) * lv.nxy, 0,
                     c.z + 1 < lv.nz ? lv.nxy : -(lv.nz - 1) * lv.nxy};
  v[0] = e[r];
#pragma unroll
  for (int i = 1; i < NQ; ++i) v[i] = e[r + ox[CX[i] + 1] + oy[CY[i] + 1] + oz[CZ[i] + 1]];
}

// The same for a level in global memory (not LDS): each load is a 32-bit
// lane offset on the array's wave-uniform base.
template <class T>
__device__ __forceinline__ void gather_lv_g(const MgLevel &lv, const Coords &c, int r,
                                            const T *__restrict__ e, T (&v)[NQ]) {
  const int ox[3] = {c.x > 0 ? -1 : lv.nx - 1, 0, c.x + 1 < lv.nx ? 1 : 1 - lv.nx};
  const int oy[3] = {c.y > 0 ? -lv.nx : (lv.ny - 1) * lv.nx, 0,
                     c.y + 1 < lv.ny ? lv.nx : -(lv.ny - 1) * lv.nx};
  const int oz[3] = {c.z > 0 ? -lv.nxy : (lv.nz - 1) * lv.nxy, 0,
                     c.z + 1 < lv.nz ? lv.nxy : -(lv.nz - 1) * lv.nxy};
  v[0] = ld32(e, (uint32_t)r);
#pragma unroll
  for (int i = 1; i < NQ; ++i)
    v[i] = ld32(e, (uint32_t)(r + ox[CX[i] + 1] + oy[CY[i] + 1] + oz[CZ[i] + 1]));
}

// Weights of a fluid cell's links that do not map it onto itself, from two
// popcounts of its flag word (links 1-6 carry W1, links 7-18 W2): all of
// them (live) or those towards a solid cell (wall).
template <class T>
__device__ __forceinline__ T link_weight(uint32_t bits) {
  return T(W1) * T(__popc(bits & 0x3Fu)) + T(W2) * T(__popc(bits & 0x3FFC0u));
}

// The stencil's diagonal at a fluid cell, sum_i w_i s_i over the non-self
// links (s_i = wall towards a solid cell, 1 otherwise).  Every kernel that
// needs it takes it from here, so that a first sweep taken by another kernel
// matches k_jacobi's bit for bit.
template <class T>
__device__ __forceinline__ T stencil_diag(const MgLevel &lv, uint32_t m) {
  const uint32_t live = ~lv.selfm & 0x3FFFFu;
  return link_weight<T>(live) + T(lv.wall - 1.0) * link_weight<T>(m & live);
}

// A correction is exactly zero at every solid cell on every level: each
// kernel that writes one writes T(0) there (or leaves the zero in place).
// So in the sums below the wall factor s_i only ever multiplies a zero
// neighbour value, and a link towards a solid cell needs no select of its
// own: the sums run over the plain weights w_i and the wall's extra
// (s_i - 1) w_i e enters once, through the flag word.

// A e at a fluid cell from its gathered correction values v, in the level's
// units: (6/h^2) sum_i w_i s_i (e - e_i), as differences (accurate when e is
// smooth), with e_i = 0 towards a solid cell.
template <class T>
__device__ __forceinline__ T apply_A_v(const MgLevel &lv, uint32_t m, const T (&v)[NQ]) {
  T acc = T(0);
#pragma unroll
  for (int i = 1; i < NQ; ++i) {
    if ((lv.selfm >> (i - 1)) & 1u) continue;
    acc += T(WQ[i]) * (v[0] - v[i]);
  }
  const uint32_t live = ~lv.selfm & 0x3FFFFu;
  acc += (T(lv.wall - 1.0) * link_weight<T>(m & live)) * v[0];
  return T(6.0) * T(lv.inv_h2) * acc;
}

template <class T>
__device__ __forceinline__ T apply_A(const MgLevel &lv, int r, uint32_t m, const Coords &c,
                                     const T *__restrict__ e) {
  T v[NQ];
  gather_lv(lv, c, r, e, v);
  return apply_A_v(lv, m, v);
}

// The kernels below issue a cell's neighbour loads together with its flag
// word and pick the result by the flag afterwards, so the two memory round
// trips overlap instead of following each other.

// A correction that starts at zero makes the first damped Jacobi sweep
// pointwise: at a fluid cell the neighbour sum vanishes and
// x = omega hs rhs / sum_i w_i s_i.  With jac > 0 the kernels that write a
// level's right-hand side (the restriction, the Krylov update) write that
// sweep (the value k_jacobi computes from x_in = 0) instead of zero.
template <class T>
__device__ __forceinline__ T coarse_start(const MgLevel &lv, uint32_t m, T rr, T jac, T hs) {
  if (jac == T(0) || (m & SOLID_BIT)) return T(0);
  return jac * ((hs * rr) / stencil_diag<T>(lv, m));
}

// ---- outer residual (FP64) ----------------------------------------------------

template <class T>
__global__ __launch_bounds__(BLOCK) void k_outer_resid(MgLevel lv, const uint32_t *__restrict__ mask,
                                                       const double *__restrict__ src,
                                                       const double *__restrict__ phi,
                                                       T *__restrict__ r0, T *__restrict__ e0,
                                                       double *__restrict__ partial,
                                                       const SolveCtl *__restrict__ ctl,
                                                       double *__restrict__ r64,
                                                       KrylovCtl *__restrict__ kc, T jacobi) {
  __shared__ double sm[BLOCK / WAVE];
  if (ctl->done) return;
  const int lb = xcd_block(blockIdx.x, gridDim.x, BLOCK, lv.nxy, lv.xcd);
  const int r = lb * BLOCK + threadIdx.x;
  if (kc && r == 0) kc->first = 1;  // a new Krylov sequence starts from this residual
  double a = 0.0;
  if (r < lv.n) {
    const Coords c = coords_of(r, lv);
    double pn[NQ];
    gather_lv_g(lv, c, r, phi, pn);
    const double sr = src[r];
    const uint32_t m = mask[r];
    // the potential itself, not a correction: solid neighbours hold the
    // electrode's value, so each wall link takes its factor here
    double acc = 0.0;
#pragma unroll
    for (int i = 1; i < NQ; ++i) {
      if ((lv.selfm >> (i - 1)) & 1u) continue;
      const double ws = solid_link(m, i) ? lv.wall * WQ[i] : WQ[i];
      acc += ws * (pn[i] - pn[0]);
    }
    const double R = (m & SOLID_BIT) ? 0.0 : 6.0 * (acc + sr);
    a = fabs(R);
    const T rr = T(R);
    r0[r] = rr;
    // the correction starts at 0; with jacobi > 0 the V-cycle's first Jacobi
    // sweep, which from 0 is pointwise, is taken here (the arithmetic of
    // k_jacobi with every neighbour value 0)
    T e = T(0);
    if (jacobi > T(0) && !(m & SOLID_BIT)) {
      const T num = T(lv.h2 / 6.0) * rr;  // the neighbour sum is +0
      e = T(0) + jacobi * (num / stencil_diag<T>(lv, m) - T(0));
    }
    e0[r] = e;
    if (r64) r64[r] = R;
  }
  a = block_max(a, sm);
  if (threadIdx.x == 0) partial[lb] = a;
}

// ---- the stencil kernels on plane rings (see lbe_device.h) ---------------------

// The residual check of k_outer_resid on a ring of phi.  The maximum over a
// block's cells does not depend on which cells a block takes.
template <class T>
__global__ __launch_bounds__(BLOCK) void k_outer_resid_ring(
    MgLevel lv, const uint32_t *__restrict__ mask, const double *__restrict__ src,
    const double *__restrict__ phi, T *__restrict__ r0, T *__restrict__ e0,
    double *__restrict__ partial, const SolveCtl *__restrict__ ctl, double *__restrict__ r64,
    KrylovCtl *__restrict__ kc, T jacobi, int zrun) {
  __shared__ double ring[4][RING_HP];
  __shared__ double sm[BLOCK / WAVE];
  if (ctl->done) return;
  const RingTile t = ring_tile(lv, zrun);
  if (kc && t.lb == 0 && threadIdx.x == 0) kc->first = 1;  // a new Krylov sequence
  PlaneRing<double> pr;
  ring_start(lv, t, pr, ring, phi);
  uint32_t rn = t.rxy + (uint32_t)lv.nxy * (uint32_t)t.z0;
  uint32_t m_next = ld32(mask, rn);
  double s_next = ld32(src, rn);
  double a = 0.0;
  for (int z = t.z0; z < t.zend; ++z) {
    const int r = (int)rn;
    const uint32_t m = m_next;
    const double sr = s_next;
    ring_advance(lv, t, z, pr, ring, phi);
    if (z + 1 < t.zend) {
      rn += (uint32_t)lv.nxy;
      m_next = ld32(mask, rn);
      s_next = ld32(src, rn);
    }
    __syncthreads();
    double pn[NQ];
    ring_gather(t, z, ring, pn);
    double acc = 0.0;
#pragma unroll
    for (int i = 1; i < NQ; ++i) {
      if ((lv.selfm >> (i - 1)) & 1u) continue;
      const double ws = solid_link(m, i) ? lv.wall * WQ[i] : WQ[i];
      acc += ws * (pn[i] - pn[0]);
    }
    const double R = (m & SOLID_BIT) ? 0.0 : 6.0 * (acc + sr);
    a = nanmax(a, fabs(R));
    const T rr = T(R);
    r0[r] = rr;
    T e = T(0);
    if (jacobi > T(0) && !(m & SOLID_BIT)) {
      const T num = T(lv.h2 / 6.0) * rr;
      e = T(0) + jacobi * (num / stencil_diag<T>(lv, m) - T(0));
    }
    e0[r] = e;
    if (r64) r64[r] = R;
  }
  a = block_max(a, sm);
  if (threadIdx.x == 0) partial[t.lb] = a;
}

// ---- flexible conjugate gradients around the V-cycle -------------------------
// The V-cycle is a fixed but non-symmetric preconditioner (mean restriction is
// not the transpose of the mirrored prolongation, and the mixed form applies it
// in FP32), so directions are A-orthogonalised against the previous one only
// (flexible CG with one stored direction).  All scalars stay on the device.

// One iteration takes two passes over the finest level.  The new direction
// is p = z + beta p' (z: the V-cycle's output for the current residual r; p',
// q' = A p': the previous direction and its image), so its image needs no
// stencil of its own: q = A z + beta q'.  The first pass forms A z and the
// sums (z, q'), (z, A z), (r, z), (r, p'); from them, with beta = -(z, q') /
// (p', q'), follow (p, q) = (z, A z) + 2 beta (z, q') + beta^2 (p', q') and
// (r, p) = (r, z) + beta (r, p'), hence alpha = (r, p) / (p, q) (one small
// kernel).  The second pass writes p and q, moves phi by alpha p and r by
// -alpha q, and checks the residual.

template <class T>
__global__ __launch_bounds__(BLOCK) void k_fcg_az(MgLevel lv, const uint32_t *__restrict__ mask,
                                                  const T *__restrict__ z,
                                                  const T *__restrict__ q_prev,
                                                  const T *__restrict__ p_prev,
                                                  const double *__restrict__ rv,
                                                  double *__restrict__ az,
                                                  double *__restrict__ partial,
                                                  const SolveCtl *__restrict__ ctl) {
  __shared__ double sm[BLOCK / WAVE];
  if (ctl->done) return;
  const int lb = xcd_block(blockIdx.x, gridDim.x, BLOCK, lv.nxy, lv.xcd);
  const int r = lb * BLOCK + threadIdx.x;
  double zq = 0.0, zaz = 0.0, rz = 0.0, rp = 0.0;
  if (r < lv.n) {
    const Coords c = coords_of(r, lv);
    T v[NQ];
    gather_lv_g(lv, c, r, z, v);
    const uint32_t m = mask[r];
    double a = 0.0;  // a solid cell stores its zero too: whole cache lines
    if (!(m & SOLID_BIT)) {
      double vd[NQ];
#pragma unroll
      for (int i = 0; i < NQ; ++i) vd[i] = double(v[i]);
      a = apply_A_v<double>(lv, m, vd);
      const double rr = rv[r];
      zq = vd[0] * double(q_prev[r]);
      zaz = vd[0] * a;
      rz = rr * vd[0];
      rp = rr * double(p_prev[r]);
    }
    az[r] = a;
  }
  const int nb = gridDim.x;
  zq = block_sum(zq, sm);
  if (threadIdx.x == 0) partial[lb] = zq;
  zaz = block_sum(zaz, sm);
  if (threadIdx.x == 0) partial[nb + lb] = zaz;
  rz = block_sum(rz, sm);
  if (threadIdx.x == 0) partial[2 * nb + lb] = rz;
  rp = block_sum(rp, sm);
  if (threadIdx.x == 0) partial[3 * nb + lb] = rp;
}

// k_fcg_az on a ring of z.  Each thread adds its cells' terms plane by
// plane before the block sums, so the sums take another order than the
// untiled kernel's (fixed for a given lattice).
template <class T>
__global__ __launch_bounds__(BLOCK) void k_fcg_az_ring(MgLevel lv, const uint32_t *__restrict__ mask,
                                                       const T *__restrict__ z,
                                                       const T *__restrict__ q_prev,
                                                       const T *__restrict__ p_prev,
                                                       const double *__restrict__ rv,
                                                       double *__restrict__ az,
                                                       double *__restrict__ partial,
                                                       const SolveCtl *__restrict__ ctl,
                                                       int zrun) {
  __shared__ T ring[4][RING_HP];
  __shared__ double sm[BLOCK / WAVE];
  if (ctl->done) return;
  const RingTile t = ring_tile(lv, zrun);
  PlaneRing<T> pr;
  ring_start(lv, t, pr, ring, z);
  uint32_t rn = t.rxy + (uint32_t)lv.nxy * (uint32_t)t.z0;
  uint32_t m_next = ld32(mask, rn);
  double q_next = double(ld32(q_prev, rn)), p_next = double(ld32(p_prev, rn));
  double r_next = ld32(rv, rn);
  double zq = 0.0, zaz = 0.0, rz = 0.0, rp = 0.0;
  for (int zp = t.z0; zp < t.zend; ++zp) {
    const int r = (int)rn;
    const uint32_t m = m_next;
    const double qv = q_next, pv = p_next, rr = r_next;
    ring_advance(lv, t, zp, pr, ring, z);
    if (zp + 1 < t.zend) {
      rn += (uint32_t)lv.nxy;
      m_next = ld32(mask, rn);
      q_next = double(ld32(q_prev, rn));
      p_next = double(ld32(p_prev, rn));
      r_next = ld32(rv, rn);
    }
    __syncthreads();
    T v[NQ];
    ring_gather(t, zp, ring, v);
    double a = 0.0;  // a solid cell stores its zero too: whole cache lines
    if (!(m & SOLID_BIT)) {
      double vd[NQ];
#pragma unroll
      for (int i = 0; i < NQ; ++i) vd[i] = double(v[i]);
      a = apply_A_v<double>(lv, m, vd);
      zq += vd[0] * qv;
      zaz += vd[0] * a;
      rz += rr * vd[0];
      rp += rr * pv;
    }
    az[r] = a;
  }
  const int nb = gridDim.x;
  zq = block_sum(zq, sm);
  if (threadIdx.x == 0) partial[t.lb] = zq;
  zaz = block_sum(zaz, sm);
  if (threadIdx.x == 0) partial[nb + t.lb] = zaz;
  rz = block_sum(rz, sm);
  if (threadIdx.x == 0) partial[2 * nb + t.lb] = rz;
  rp = block_sum(rp, sm);
  if (threadIdx.x == 0) partial[3 * nb + t.lb] = rp;
}

// The four sums of k_fcg_az's partials in one pass (their loads in flight
// together), each combined in a fixed order.
__global__ __launch_bounds__(FINAL) void k_fcg_coef(const double *__restrict__ partial, int nb,
                                                    KrylovCtl *__restrict__ kc,
                                                    const SolveCtl *__restrict__ ctl) {
  __shared__ double tree[4][FINAL];
  if (ctl->done) return;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nb; b += FINAL)
#pragma unroll
    for (int k = 0; k < 4; ++k) a[k] += partial[k * nb + b];
#pragma unroll
  for (int k = 0; k < 4; ++k) tree[k][threadIdx.x] = a[k];
  __syncthreads();
  for (int h = FINAL / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h)
#pragma unroll
      for (int k = 0; k < 4; ++k) tree[k][threadIdx.x] += tree[k][threadIdx.x + h];
    __syncthreads();
  }
  const double zq = tree[0][0], zaz = tree[1][0], rz = tree[2][0], rp_prev = tree[3][0];
  if (threadIdx.x == 0) {
    // a new sequence (first) starts from p = z
    const bool fresh = kc->first || kc->pq_prev == 0.0;
    const double beta = fresh ? 0.0 : -zq / kc->pq_prev;
    const double pq = fresh ? zaz : zaz + beta * (2.0 * zq + beta * kc->pq_prev);
    const double rp = fresh ? rz : rz + beta * rp_prev;
    kc->beta = beta;
    kc->alpha = pq > 0.0 ? rp / pq : 0.0;
    kc->pq_prev = pq;
    kc->first = 0;
  }
}

// z may be the buffer e0 points to (the V-cycle's output on the finest
// level): each site reads its z before writing its e0, so neither is
// declared __restrict__.
template <class T>
__global__ __launch_bounds__(BLOCK) void k_fcg_update(int n, const uint32_t *__restrict__ mask,
                                                      const T *z,
                                                      const double *__restrict__ az,
                                                      T *__restrict__ p,
                                                      T *__restrict__ q,
                                                      double *__restrict__ phi,
                                                      double *__restrict__ rv,
                                                      T *__restrict__ r0, T *e0,
                                                      double *__restrict__ partial,
                                                      const KrylovCtl *__restrict__ kc,
                                                      const SolveCtl *__restrict__ ctl,
                                                      MgLevel lv, T jac, T hs) {
  __shared__ double sm[BLOCK / WAVE];
  if (ctl->done) return;
  const int r = blockIdx.x * BLOCK + threadIdx.x;
  double a = 0.0;
  if (r < n) {
    double R = 0.0;
    const uint32_t m = mask[r];
    // Every cell stores p, q, phi and r, so each store writes whole cache
    // lines: a solid cell its zeros (p, q, r hold zeros there) and its
    // potential, the electrode's, unchanged.
    const bool solid = m & SOLID_BIT;
    const double beta = kc->beta, alpha = kc->alpha;
    const double zr = solid ? 0.0 : double(z[r]);
    // the directions are stored in the correction's precision, and phi and r
    // move along the stored vectors
    const T pt = T(solid ? 0.0 : (beta == 0.0 ? zr : zr + beta * double(p[r])));
    const T qt = T(solid ? 0.0 : (beta == 0.0 ? az[r] : az[r] + beta * double(q[r])));
    p[r] = pt;
    q[r] = qt;
    const double pr = double(pt), qr = double(qt);
    const double ph = phi[r];
    phi[r] = solid ? ph : ph + alpha * pr;
    R = solid ? 0.0 : rv[r] - alpha * qr;
    rv[r] = R;
    a = fabs(R);
    const T rr = T(R);
    r0[r] = rr;
    e0[r] = coarse_start<T>(lv, m, rr, jac, hs);
  }
  a = block_max(a, sm);
  if (threadIdx.x == 0) partial[blockIdx.x] = a;
}

// ---- smoother: one colour of Gauss-Seidel / SOR on A e = r ------------------

template <class T>
__global__ __launch_bounds__(BLOCK) void k_smooth(MgLevel lv, T omega, int colour, int hx, int hy,
                                                  const uint32_t *__restrict__ mask,
                                                  const T *__restrict__ rhs, T *__restrict__ e,
                                                  const SolveCtl *__restrict__ ctl) {
  if (ctl->done) return;
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
  T v[NQ];
  gather_lv(lv, c, r, (const T *)e, v);
  const T rr = rhs[r];
  T num = T(0);
#pragma unroll
  for (int i = 1; i < NQ; ++i) {
    if ((lv.selfm >> (i - 1)) & 1u) continue;
    num += T(WQ[i]) * v[i];
  }
  const T den = stencil_diag<T>(lv, m);
  num += T(lv.h2 / 6.0) * rr;
  e[r] = (T(1) - omega) * v[0] + omega * (num / den);
}

// ---- damped Jacobi sweep (one launch, every cell in parallel) --------------
// x_out = x_in + omega ([sum_i w_i s_i x_in(r+c_i) + hs rhs] / sum_i w_i s_i - x_in)

// With ADD_PHI (the last sweep of a V-cycle on the finest level), the result
// is also added to phi_add on fluid cells, as k_correct does (a kernel of its
// own name, so that profiles tell the two apart).
template <class T, bool ADD_PHI>
__global__ __launch_bounds__(BLOCK) void k_jacobi(MgLevel lv, T omega, T hs,
                                                  const uint32_t *__restrict__ mask,
                                                  const T *__restrict__ rhs,
                                                  const T *__restrict__ x_in,
                                                  T *__restrict__ x_out,
                                                  const SolveCtl *__restrict__ ctl,
                                                  double *__restrict__ phi_add) {
  if (ctl->done) return;
  const int r = blockIdx.x * BLOCK + threadIdx.x;
  if (r >= lv.n) return;
  const Coords c = coords_of(r, lv);
  T v[NQ];
  gather_lv_g(lv, c, r, x_in, v);
  const T rr = rhs[r];
  const uint32_t m = mask[r];
  T num = T(0);
#pragma unroll
  for (int i = 1; i < NQ; ++i) {
    if ((lv.selfm >> (i - 1)) & 1u) continue;
    num += T(WQ[i]) * v[i];
  }
  const T den = stencil_diag<T>(lv, m);
  num += hs * rr;
  const T xr = v[0];
  const bool solid = m & SOLID_BIT;
  const T res = solid ? T(0) : xr + omega * (num / den - xr);
  x_out[r] = res;
  // every cell, so that the store writes whole lines (a solid cell adds 0 to
  // its electrode potential)
  if (ADD_PHI) phi_add[r] += double(res);
}

// k_jacobi on a ring of x_in: the same values and arithmetic per cell.
template <class T, bool ADD_PHI>
__global__ __launch_bounds__(BLOCK) void k_jacobi_ring(MgLevel lv, T omega, T hs,
                                                       const uint32_t *__restrict__ mask,
                                                       const T *__restrict__ rhs,
                                                       const T *__restrict__ x_in,
                                                       T *__restrict__ x_out,
                                                       const SolveCtl *__restrict__ ctl,
                                                       double *__restrict__ phi_add, int zrun) {
  __shared__ T ring[4][RING_HP];
  if (ctl->done) return;
  const RingTile t = ring_tile(lv, zrun);
  PlaneRing<T> pr;
  ring_start(lv, t, pr, ring, x_in);
  uint32_t rn = t.rxy + (uint32_t)lv.nxy * (uint32_t)t.z0;
  uint32_t m_next = ld32(mask, rn);
  T r_next = ld32(rhs, rn);
  for (int z = t.z0; z < t.zend; ++z) {
    const int r = (int)rn;
    const uint32_t m = m_next;
    const T rr = r_next;
    ring_advance(lv, t, z, pr, ring, x_in);
    if (z + 1 < t.zend) {
      rn += (uint32_t)lv.nxy;
      m_next = ld32(mask, rn);
      r_next = ld32(rhs, rn);
    }
    __syncthreads();
    T v[NQ];
    ring_gather(t, z, ring, v);
    T num = T(0);
#pragma unroll
    for (int i = 1; i < NQ; ++i) {
      if ((lv.selfm >> (i - 1)) & 1u) continue;
      num += T(WQ[i]) * v[i];
    }
    const T den = stencil_diag<T>(lv, m);
    num += hs * rr;
    const T xr = v[0];
    const bool solid = m & SOLID_BIT;
    const T res = solid ? T(0) : xr + omega * (num / den - xr);
    x_out[r] = res;
    if (ADD_PHI) phi_add[r] += double(res);
  }
}

// ---- restriction: coarse rhs = mean of the fluid children's residuals -------
// Each lane evaluates one fine-cell residual.  On narrow levels eight
// consecutive lanes take the eight children of one coarse cell (lane bits =
// dx, dy, dz) and combine them with cross-lane adds (groups of eight never
// straddle a wavefront); on wide levels k_restrict_tiled keeps the lanes in
// row order and combines through LDS, in the same order.

// Residual of child j (bits dx, dy, dz) of coarse cell R, or nothing when
// the child is solid or falls outside an odd-sized fine level.
template <class T>
__device__ __forceinline__ void restrict_child(const MgTransfer &tr, int R, int j,
                                               const uint32_t *__restrict__ mf,
                                               const T *__restrict__ rf,
                                               const T *__restrict__ ef, T &v, int &cnt) {
  const Coords C = coords_of(R, tr.c);
  const int xp = 2 * C.x + (j & 1), yp = 2 * C.y + ((j >> 1) & 1), zp = 2 * C.z + (j >> 2);
  const bool inside = xp < tr.f.nx && yp < tr.f.ny && zp < tr.f.nz;
  // a child beyond an odd-sized level reads a valid cell and is dropped
  Coords c;
  c.x = wrapi(min(xp, tr.f.nx - 1) + tr.ox, tr.f.nx);
  c.y = wrapi(min(yp, tr.f.ny - 1) + tr.oy, tr.f.ny);
  c.z = wrapi(min(zp, tr.f.nz - 1) + tr.oz, tr.f.nz);
  const int r = c.x + tr.f.nx * (c.y + tr.f.ny * c.z);
  T e[NQ];
  gather_lv(tr.f, c, r, ef, e);  // also on LDS levels (k_mg_small)
  const T rr = rf[r];
  const uint32_t m = mf[r];
  const T res = rr - apply_A_v<T>(tr.f, m, e);
  if (inside && !(m & SOLID_BIT)) {
    v = res;
    cnt = 1;
  }
}

// sum of v and cnt over the eight lanes of an aligned group
template <class T>
__device__ __forceinline__ void group8_sum(T &v, int &cnt) {
#pragma unroll
  for (int off = 1; off < 8; off <<= 1) {
    v += __shfl_xor(v, off);
    cnt += __shfl_xor(cnt, off);
  }
}

template <class T>
__global__ __launch_bounds__(BLOCK) void k_restrict(MgTransfer tr, const uint32_t *__restrict__ mf,
                                                    const uint32_t *__restrict__ mc,
                                                    const T *__restrict__ rf,
                                                    const T *__restrict__ ef, T *__restrict__ rc,
                                                    T *__restrict__ ec,
                                                    const SolveCtl *__restrict__ ctl, T jac,
                                                    T hs) {
  if (ctl->done) return;
  const int t = blockIdx.x * BLOCK + threadIdx.x;
  const int R = t >> 3, j = t & 7;
  T v = T(0);
  int cnt = 0;
  bool fluid = false;
  uint32_t m = SOLID_BIT;
  if (R < tr.c.n) {
    restrict_child<T>(tr, R, j, mf, rf, ef, v, cnt);
    m = mc[R];
    fluid = !(m & SOLID_BIT);
    if (!fluid) {
      v = T(0);
      cnt = 0;
    }
  }
  group8_sum(v, cnt);
  if (j == 0 && R < tr.c.n) {
    const T rv = (fluid && cnt) ? v / T(cnt) : T(0);
    rc[R] = rv;
    ec[R] = coarse_start<T>(tr.c, m, rv, jac, hs);
  }
}

// The same restriction with one fine cell per thread in row order: a block
// takes a tile of 16 x 2 x 1 coarse cells, i.e. 32 x 4 x 2 fine cells, so
// the lanes of a wave read 32 consecutive fine cells of two rows (whole
// cache lines) instead of 2 x 2 x 2 blocks; the eight children of a coarse
// cell then meet in LDS and are summed in the eight-lane tree's order, so
// every sum is bit for bit that of k_restrict.
constexpr int RT_X = 16, RT_Y = 2;  // coarse cells per tile along x and y

template <class T>
__global__ __launch_bounds__(BLOCK) void k_restrict_tiled(MgTransfer tr,
                                                          const uint32_t *__restrict__ mf,
                                                          const uint32_t *__restrict__ mc,
                                                          const T *__restrict__ rf,
                                                          const T *__restrict__ ef,
                                                          T *__restrict__ rc, T *__restrict__ ec,
                                                          const SolveCtl *__restrict__ ctl, T jac,
                                                          T hs) {
  static_assert(2 * RT_X * 2 * RT_Y * 2 == BLOCK, "one fine cell per thread");
  __shared__ T sv[BLOCK];
  __shared__ int sc[BLOCK];
  if (ctl->done) return;
  const int bx = blockIdx.x, by = blockIdx.y, bz = blockIdx.z;
  const int t = threadIdx.x;
  const int fx = t & (2 * RT_X - 1), fy = (t / (2 * RT_X)) & (2 * RT_Y - 1), fz = t / (4 * RT_X * RT_Y);
  const int X = bx * RT_X + (fx >> 1), Y = by * RT_Y + (fy >> 1), Z = bz;
  T v = T(0);
  int cnt = 0;
  if (X < tr.c.nx && Y < tr.c.ny) {
    const int R = X + tr.c.nx * (Y + tr.c.ny * Z);
    if (!(mc[R] & SOLID_BIT))
      restrict_child<T>(tr, R, (fx & 1) | ((fy & 1) << 1) | (fz << 2), mf, rf, ef, v, cnt);
  }
  sv[t] = v;
  sc[t] = cnt;
  __syncthreads();
  if (t >= RT_X * RT_Y) return;
  const int cx = t % RT_X, cy = t / RT_X;
  const int Xo = bx * RT_X + cx, Yo = by * RT_Y + cy;
  if (Xo >= tr.c.nx || Yo >= tr.c.ny) return;
  // child (a, b, d) of coarse cell (cx, cy) sits at thread
  // (2 cx + a) + 2 RT_X (2 cy + b) + 4 RT_X RT_Y d
  const int base = 2 * cx + 2 * RT_X * (2 * cy);
  T q[8];
  int n[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k = base + (j & 1) + 2 * RT_X * ((j >> 1) & 1) + 4 * RT_X * RT_Y * (j >> 2);
    q[j] = sv[k];
    n[j] = sc[k];
  }
  const T sum = ((q[0] + q[1]) + (q[2] + q[3])) + ((q[4] + q[5]) + (q[6] + q[7]));
  const int cn = ((n[0] + n[1]) + (n[2] + n[3])) + ((n[4] + n[5]) + (n[6] + n[7]));
  const int R = Xo + tr.c.nx * (Yo + tr.c.ny * bz);
  const uint32_t m = mc[R];
  const bool fluid = !(m & SOLID_BIT);
  const T rv = (fluid && cn) ? sum / T(cn) : T(0);
  rc[R] = rv;
  ec[R] = coarse_start<T>(tr.c, m, rv, jac, hs);
}

// The restriction on a ring of the fine correction.  A tile starts at the
// transfer's offsets, so the children of a coarse cell are lanes 2k, 2k + 1
// of a row (dx), the same lanes of the next row, 32 lanes on (dy), and two
// consecutive planes of a run (dz); their residuals are summed in that
// order, which is k_restrict's eight-lane tree, so the results are its bits.
template <class T>
__global__ __launch_bounds__(BLOCK) void k_restrict_ring(MgTransfer tr,
                                                         const uint32_t *__restrict__ mf,
                                                         const uint32_t *__restrict__ mc,
                                                         const T *__restrict__ rf,
                                                         const T *__restrict__ ef,
                                                         T *__restrict__ rc, T *__restrict__ ec,
                                                         const SolveCtl *__restrict__ ctl, T jac,
                                                         T hs, int zrun) {
  __shared__ T ring[4][RING_HP];
  if (ctl->done) return;
  const MgLevel &lv = tr.f;
  const RingTile t = ring_tile(lv, zrun, tr.ox, tr.oy, tr.oz);
  PlaneRing<T> pr;
  ring_start(lv, t, pr, ring, ef);
  const int lane = threadIdx.x & (WAVE - 1);
  const int lx = threadIdx.x % RING_TX, ly = threadIdx.x / RING_TX;
  // the coarse cell of this thread's children pair along x and y
  const int X = (t.x0 - tr.ox + lx) >> 1, Y = (t.y0 - tr.oy + ly) >> 1;
  const bool writer = !(lane & 1) && !(lane & RING_TX);
  uint32_t rn = t.rxy + (uint32_t)lv.nxy * (uint32_t)wrapi(t.z0, lv.nz);
  uint32_t m_next = ld32(mf, rn);
  T r_next = ld32(rf, rn);
  T s_lo = T(0);
  int c_lo = 0;
  for (int z = t.z0; z < t.zend; ++z) {
    const uint32_t m = m_next;
    const T rr = r_next;
    ring_advance(lv, t, z, pr, ring, ef);
    if (z + 1 < t.zend) {
      rn = t.rxy + (uint32_t)lv.nxy * (uint32_t)wrapi(z + 1, lv.nz);
      m_next = ld32(mf, rn);
      r_next = ld32(rf, rn);
    }
    __syncthreads();
    T e[NQ];
    ring_gather(t, z, ring, e);
    T v = T(0);
    int cnt = 0;
    if (!(m & SOLID_BIT)) {
      v = rr - apply_A_v<T>(lv, m, e);
      cnt = 1;
    }
    v += __shfl_xor(v, 1);  // dx
    cnt += __shfl_xor(cnt, 1);
    v += __shfl_xor(v, RING_TX);  // dy
    cnt += __shfl_xor(cnt, RING_TX);
    if (!((z - t.z0) & 1)) {  // dz = 0
      s_lo = v;
      c_lo = cnt;
      continue;
    }
    if (writer) {
      const T sum = s_lo + v;
      const int cn = c_lo + cnt;
      const int Z = (z - tr.oz) >> 1;
      const int R = X + tr.c.nx * (Y + tr.c.ny * Z);
      const uint32_t mcr = mc[R];
      const T rv = (!(mcr & SOLID_BIT) && cn) ? sum / T(cn) : T(0);
      rc[R] = rv;
      ec[R] = coarse_start<T>(tr.c, mcr, rv, jac, hs);
    }
  }
}

// ---- prolongation: e_f += trilinear interpolation of e_c --------------------

// trilinear interpolation of e_c at fine cell r (mirrored across solid cells)
template <class T>
__device__ __forceinline__ T prolong_value(const MgTransfer &tr, int r,
                                           const uint32_t *__restrict__ mc,
                                           const T *__restrict__ ec) {
  const Coords c = coords_of(r, tr.f);
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
  // flags and corrections of the eight surrounding coarse cells (k = 0 is the
  // parent), loaded together before use
  uint32_t mk[8];
  T ev[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int ix = (k & 1) ? Nb[0] : P[0];
    const int iy = (k & 2) ? Nb[1] : P[1];
    const int iz = (k & 4) ? Nb[2] : P[2];
    const int R = ix + tr.c.nx * (iy + tr.c.ny * iz);
    mk[k] = mc[R];
    ev[k] = ec[R];
  }
  if (mk[0] & SOLID_BIT) return T(0);
  // value beyond a wall: mirrored (-e) when the wall lies on the cell face
  // (factor 2), zero when it lies on the solid cell (first-order scheme)
  const T ep = tr.c.wall > 1.5 ? -ev[0] : T(0);
  T v = T(0);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const T w = ((k & 1) ? T(1) - wgt[0] : wgt[0]) * ((k & 2) ? T(1) - wgt[1] : wgt[1]) *
                ((k & 4) ? T(1) - wgt[2] : wgt[2]);
    if (w == T(0)) continue;
    const T val = (mk[k] & SOLID_BIT) ? ep : ev[k];
    v += w * val;
  }
  return v;
}

template <class T>
__global__ __launch_bounds__(BLOCK) void k_prolong(MgTransfer tr, const uint32_t *__restrict__ mf,
                                                   const uint32_t *__restrict__ mc,
                                                   const T *__restrict__ ec, T *__restrict__ ef,
                                                   const SolveCtl *__restrict__ ctl) {
  if (ctl->done) return;
  const int r = blockIdx.x * BLOCK + threadIdx.x;
  if (r >= tr.f.n) return;
  const T e0 = ef[r];
  const T pv = prolong_value<T>(tr, r, mc, ec);
  // every cell stores (a solid one its value back), so that the store
  // writes whole cache lines
  ef[r] = (mf[r] & SOLID_BIT) ? e0 : e0 + pv;
}

// The prolongation on a fine tile of RING_TX x RING_TY cells and a run of
// zrun planes (even, at most RING_PROLONG_ZRUN), starting at the transfer's
// offsets like k_restrict_ring: the coarse cells it interpolates from, a box
// of (RING_TX / 2 + 2) x (RING_TY / 2 + 2) x (zrun / 2 + 2), are loaded into
// LDS once, then each fine plane is interpolated from there with
// prolong_value's arithmetic (same bits).
constexpr int RING_PROLONG_ZRUN = 16;
constexpr int PR_CX = RING_TX / 2 + 2, PR_CY = RING_TY / 2 + 2, PR_CP = PR_CX * PR_CY;
constexpr int PR_CZ = RING_PROLONG_ZRUN / 2 + 2;

template <class T>
__global__ __launch_bounds__(BLOCK) void k_prolong_ring(MgTransfer tr, const uint32_t *__restrict__ mf,
                                                        const uint32_t *__restrict__ mc,
                                                        const T *__restrict__ ec,
                                                        T *__restrict__ ef,
                                                        const SolveCtl *__restrict__ ctl,
                                                        int zrun) {
  __shared__ T cv[PR_CZ][PR_CP];
  __shared__ uint32_t cs[PR_CZ][PR_CP];
  if (ctl->done) return;
  const MgLevel &f = tr.f, &c = tr.c;
  const RingTile t = ring_tile(f, zrun, tr.ox, tr.oy, tr.oz);
  // the coarse box: parents of the tile's cells and one cell around them
  const int X0 = (t.x0 - tr.ox) / 2 - 1, Y0 = (t.y0 - tr.oy) / 2 - 1, Z0 = (t.z0 - tr.oz) / 2 - 1;
  const int ncp = (t.zend - t.z0) / 2 + 2;
  for (int i = threadIdx.x; i < ncp * PR_CP; i += BLOCK) {
    const int pz = i / PR_CP, rem = i - pz * PR_CP, py = rem / PR_CX, px = rem - py * PR_CX;
    const int R = wrapi(X0 + px, c.nx) + c.nx * (wrapi(Y0 + py, c.ny) + c.ny * wrapi(Z0 + pz, c.nz));
    cv[pz][rem] = ec[R];
    cs[pz][rem] = mc[R] & SOLID_BIT;
  }
  const int lx = threadIdx.x % RING_TX, ly = threadIdx.x / RING_TX;
  // parent and nearer neighbour in the box along x and y
  const int P0 = (lx >> 1) + 1, N0 = P0 + ((lx & 1) ? 1 : -1);
  const int P1 = (ly >> 1) + 1, N1 = P1 + ((ly & 1) ? 1 : -1);
  const T wgt = T(0.75);
  uint32_t rn = t.rxy + (uint32_t)f.nxy * (uint32_t)wrapi(t.z0, f.nz);
  T e_next = ld32(ef, rn);
  uint32_t m_next = ld32(mf, rn);
  __syncthreads();
  for (int z = t.z0; z < t.zend; ++z) {
    const uint32_t r = rn;
    const T e0 = e_next;
    const uint32_t m = m_next;
    if (z + 1 < t.zend) {
      rn = t.rxy + (uint32_t)f.nxy * (uint32_t)wrapi(z + 1, f.nz);
      e_next = ld32(ef, rn);
      m_next = ld32(mf, rn);
    }
    const int fz = z - t.z0;
    const int P2 = (fz >> 1) + 1, N2 = P2 + ((fz & 1) ? 1 : -1);
    T pv = T(0);
    if (!cs[P2][P0 + PR_CX * P1]) {
      const T ev0 = cv[P2][P0 + PR_CX * P1];
      const T ep = c.wall > 1.5 ? -ev0 : T(0);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const T w = ((k & 1) ? T(1) - wgt : wgt) * ((k & 2) ? T(1) - wgt : wgt) *
                    ((k & 4) ? T(1) - wgt : wgt);
        const int i = ((k & 1) ? N0 : P0) + PR_CX * ((k & 2) ? N1 : P1);
        const int pz = (k & 4) ? N2 : P2;
        const T val = cs[pz][i] ? ep : cv[pz][i];
        pv += w * val;
      }
    }
    st32(ef, r, (m & SOLID_BIT) ? e0 : e0 + pv);
  }
}

// ---- coarsest level: one work-group, sweeps with barriers ----------------------
// Jacobi in pairs through e2 (jacobi > 0, the level needs no colouring) or
// four-colour Gauss-Seidel with relaxation omega.

template <class T>
__global__ __launch_bounds__(COARSE_BLOCK) void k_coarse(MgLevel lv, T omega, T jacobi, int sweeps,
                                                         const uint32_t *__restrict__ mask,
                                                         const T *__restrict__ rhs,
                                                         T *__restrict__ e, T *__restrict__ e2,
                                                         const SolveCtl *__restrict__ ctl) {
  if (ctl->done) return;
  const T hs = T(lv.h2 / 6.0);
  if (jacobi > T(0)) {
    for (int s = 0; s < sweeps; s += 2)
      for (int pass = 0; pass < 2; ++pass) {
        const T *xi = pass ? e2 : e;
        T *xo = pass ? e : e2;
        for (int r = threadIdx.x; r < lv.n; r += COARSE_BLOCK) {
          const uint32_t m = mask[r];
          if (m & SOLID_BIT) {
            xo[r] = T(0);
            continue;
          }
          const Coords c = coords_of(r, lv);
          T v[NQ];
          gather_lv(lv, c, r, xi, v);
          T num = T(0);
#pragma unroll
          for (int i = 1; i < NQ; ++i) {
            if ((lv.selfm >> (i - 1)) & 1u) continue;
            num += T(WQ[i]) * v[i];
          }
          const T den = stencil_diag<T>(lv, m);
          num += hs * rhs[r];
          xo[r] = v[0] + jacobi * (num / den - v[0]);
        }
        __threadfence_block();
        __syncthreads();
      }
    return;
  }
  for (int s = 0; s < sweeps; ++s) {
    for (int col = 0; col < 4; ++col) {
      for (int r = threadIdx.x; r < lv.n; r += COARSE_BLOCK) {
        const Coords c = coords_of(r, lv);
        if ((((c.x + c.z) & 1) + 2 * ((c.y + c.z) & 1)) != col) continue;
        const uint32_t m = mask[r];
        if (m & SOLID_BIT) continue;
        T num = T(0);
#pragma unroll
        for (int i = 1; i < NQ; ++i) {
          if ((lv.selfm >> (i - 1)) & 1u) continue;
          num += T(WQ[i]) * e[nbr_of(lv, c, i)];
        }
        const T den = stencil_diag<T>(lv, m);
        num += hs * rhs[r];
        e[r] = (T(1) - omega) * e[r] + omega * (num / den);
      }
      __threadfence_block();
      __syncthreads();
    }
  }
}

// ---- coarsest level, exact: e = A^-1 r over the level's fluid cells ----------
// Eight lanes per row: lane `part` sums the columns j = part (mod 8), then the
// group adds its partial sums.  The inverse is stored column-major
// (ainv[j * nf + row]).

// The exact coarsest solve e = A^-1 r over the nf fluid cells: the inverse is
// column-major (ainv[j nf + row]).  Its columns are split into P = DENSE_T /
// nf interleaved parts (column j in part j mod P); part p of a row is summed
// in column order, and the P part sums in part order.  In one work-group of
// DENSE_T threads, thread t takes row t mod nf of part t / nf, so the lanes
// of a wave read consecutive rows of one column: contiguous loads.
constexpr int DENSE_T = 1024;

template <class T>
__device__ __forceinline__ T dense_part(int nf, int parts, const T *__restrict__ ainv,
                                        const T *__restrict__ x, int row, int part) {
  T acc = T(0);
#pragma unroll 8
  for (int j = part; j < nf; j += parts) acc += ainv[(size_t)j * nf + row] * x[j];
  return acc;
}

// one thread per row, the parts in sequence: the same sums as the split
// across a work-group
template <class T>
__global__ __launch_bounds__(BLOCK) void k_coarse_dense(int nf, const T *__restrict__ ainv,
                                                        const int *__restrict__ fcell,
                                                        const T *__restrict__ rhs,
                                                        T *__restrict__ e,
                                                        const SolveCtl *__restrict__ ctl) {
  __shared__ T xc[MG_MAX_DENSE];
  if (ctl->done) return;
  for (int j = threadIdx.x; j < nf; j += BLOCK) xc[j] = rhs[fcell[j]];
  __syncthreads();
  const int row = blockIdx.x * BLOCK + threadIdx.x;
  if (row >= nf) return;
  const int parts = DENSE_T / nf;
  T v = dense_part(nf, parts, ainv, xc, row, 0);
  for (int p = 1; p < parts; ++p) v += dense_part(nf, parts, ainv, xc, row, p);
  e[fcell[row]] = v;
}

// ---- the coarse end of the V-cycle in one work-group --------------------------
// Levels S.lv[0..nlev-1] live in LDS (correction, right-hand side and flag
// word per cell).  Same arithmetic as the multi-kernel path: four-colour
// Gauss-Seidel, mean-of-children restriction, mirrored trilinear
// prolongation, exact (dense inverse) or swept coarsest level.

constexpr int SMALL_BLOCK = 1024;
static_assert(SMALL_BLOCK == DENSE_T, "the dense solve splits one work-group's threads");

// A work-group's cells of a level: the cyclic range of len cells from start
// (start 0 and the whole level for one group).
__device__ __forceinline__ int range_cell(int start, int i, int n) {
  const int r = start + i;
  return r < n ? r : r - n;
}

template <class T>
__device__ void small_smooth(const MgSmall &S, int k, int sweeps, T *lds, const uint32_t *sm,
                             int start, int len) {
  const MgLevel &lv = S.lv[k];
  T *e = lds + S.off_e[k];
  const T *rh = lds + S.off_r[k];
  const uint32_t *mk = sm + S.off_m[k];
  const T hs = T(lv.h2 / 6.0);
  if (S.jacobi > 0.0) {
    // Jacobi alternating e -> e2 -> e ..., the arithmetic of k_jacobi; an odd
    // count ends with a copy back into e
    T *e2 = lds + S.off_e2[k];
    const T om = T(S.jacobi);
    for (int s = 0; s < sweeps; ++s) {
      {
        const T *xi = (s & 1) ? e2 : e;
        T *xo = (s & 1) ? e : e2;
        for (int i = threadIdx.x; i < len; i += SMALL_BLOCK) {
          const int r = range_cell(start, i, lv.n);
          const uint32_t m = mk[r];
          if (m & SOLID_BIT) {
            xo[r] = T(0);
            continue;
          }
          const Coords c = coords_of(r, lv);
          T v[NQ];
          gather_lv(lv, c, r, xi, v);
          T num = T(0);
#pragma unroll
          for (int i = 1; i < NQ; ++i) {
            if ((lv.selfm >> (i - 1)) & 1u) continue;
            num += T(WQ[i]) * v[i];
          }
          const T den = stencil_diag<T>(lv, m);
          num += hs * rh[r];
          xo[r] = v[0] + om * (num / den - v[0]);
        }
        __syncthreads();
      }
    }
    if (sweeps & 1) {
      for (int i = threadIdx.x; i < len; i += SMALL_BLOCK) {
        const int r = range_cell(start, i, lv.n);
        e[r] = e2[r];
      }
      __syncthreads();
    }
    return;
  }
  // four-colour Gauss-Seidel
  const int hx = (lv.nx + 1) / 2, hy = (lv.ny + 1) / 2, plane = hx * hy;
  for (int s = 0; s < sweeps; ++s)
    for (int col = 0; col < 4; ++col) {
      for (int t = threadIdx.x; t < plane * lv.nz; t += SMALL_BLOCK) {
        Coords c;
        c.z = t / plane;
        const int rem = t - c.z * plane;
        const int iy = rem / hx, ix = rem - iy * hx;
        c.x = 2 * ix + ((col ^ c.z) & 1);
        c.y = 2 * iy + (((col >> 1) ^ c.z) & 1);
        if (c.x >= lv.nx || c.y >= lv.ny) continue;
        const int r = c.x + lv.nx * (c.y + lv.ny * c.z);
        if (((r - start) % lv.n + lv.n) % lv.n >= len) continue;  // another group's cell
        const uint32_t m = mk[r];
        if (m & SOLID_BIT) continue;
        T v[NQ];
        gather_lv(lv, c, r, (const T *)e, v);
        T num = T(0);
#pragma unroll
        for (int i = 1; i < NQ; ++i) {
          if ((lv.selfm >> (i - 1)) & 1u) continue;
          num += T(WQ[i]) * v[i];
        }
        const T den = stencil_diag<T>(lv, m);
        num += hs * rh[r];
        e[r] = num / den;  // Gauss-Seidel (omega = 1)
      }
      __syncthreads();
    }
}

template <class T>
__global__ __launch_bounds__(SMALL_BLOCK) void k_mg_small(MgSmall S, const T *__restrict__ r_in,
                                                          T *__restrict__ e_out,
                                                          const SolveCtl *__restrict__ ctl) {
  extern __shared__ double smem_raw[];
  if (ctl->done) return;
  T *lds = reinterpret_cast<T *>(smem_raw);
  uint32_t *sm = reinterpret_cast<uint32_t *>(smem_raw);  // flag words, offsets in 4-byte units
  // this work-group's group: a range of cells on every level (whole levels
  // when there is one group)
  const int G = S.ngroups, g = blockIdx.x;
  auto first = [&](int k) { return S.groups ? S.groups[2 * (k * G + g)] : 0; };
  auto count = [&](int k) { return S.groups ? S.groups[2 * (k * G + g) + 1] : S.lv[k].n; };
  // flags of every level; with several groups every correction and
  // right-hand side starts at zero, so that cells of other groups (never
  // written here) read as the solid cells between them
  for (int k = 0; k < S.nlev; ++k)
    for (int r = threadIdx.x; r < S.lv[k].n; r += SMALL_BLOCK) sm[S.off_m[k] + r] = S.mask[k][r];
  if (S.groups)
    for (int i = threadIdx.x; i < S.off_x; i += SMALL_BLOCK) lds[i] = T(0);
  __syncthreads();
  // rhs and zero correction of the first level
  for (int i = threadIdx.x; i < count(0); i += SMALL_BLOCK) {
    const int r = range_cell(first(0), i, S.lv[0].n);
    lds[S.off_r[0] + r] = r_in[r];
    lds[S.off_e[0] + r] = T(0);
  }
  __syncthreads();
  // down: smooth, restrict (eight lanes per coarse cell, as k_restrict)
  for (int k = 0; k + 1 < S.nlev; ++k) {
    small_smooth<T>(S, k, S.nu1, lds, sm, first(k), count(k));
    const MgTransfer &tr = S.tr[k + 1];
    const T *ef = lds + S.off_e[k];
    const T *rf = lds + S.off_r[k];
    const uint32_t *mf = sm + S.off_m[k];
    const uint32_t *mc = sm + S.off_m[k + 1];
    for (int t = threadIdx.x; t < 8 * count(k + 1); t += SMALL_BLOCK) {
      const int R = range_cell(first(k + 1), t >> 3, tr.c.n), j = t & 7;
      const bool fluid = !(mc[R] & SOLID_BIT);
      T v = T(0);
      int cnt = 0;
      if (fluid) restrict_child<T>(tr, R, j, mf, rf, ef, v, cnt);
      group8_sum(v, cnt);
      if (j == 0) {
        lds[S.off_e[k + 1] + R] = T(0);
        lds[S.off_r[k + 1] + R] = (fluid && cnt) ? v / T(cnt) : T(0);
      }
    }
    __syncthreads();
  }
  // coarsest
  {
    const int k = S.nlev - 1;
    T *e = lds + S.off_e[k];
    const T *rh = lds + S.off_r[k];
    if (S.ainv) {
      // compact right-hand side over the fluid cells, then the part sums of
      // every row (k_coarse_dense's arithmetic) through LDS; a group's rows
      // and columns are its own fluid cells (the inverse is block-diagonal
      // by group), so the columns of other groups, exact zeros, are skipped
      const T *ainv = reinterpret_cast<const T *>(S.ainv);
      // the group's rows: a cyclic range of fluid indices; its columns, in
      // increasing order, are one run or (through the wrap) two
      const int nf = S.nf;
      const int f0 = S.groups ? S.groups[2 * (S.nlev * G + g)] : 0;
      const int ng = S.groups ? S.groups[2 * (S.nlev * G + g) + 1] : nf;
      const int wrapped = f0 + ng > nf ? f0 + ng - nf : 0;  // columns [0, wrapped)
      const int f1 = f0 + ng - wrapped;                       // and [f0, f1)
      T *xc = lds + S.off_x;
      T *psum = xc + nf;  // DENSE_T entries
      for (int i = threadIdx.x; i < ng; i += SMALL_BLOCK) {
        const int j = range_cell(f0, i, nf);
        xc[j] = rh[S.fcell[j]];
      }
      __syncthreads();
      const int parts = DENSE_T / nf;
      if (ng > 0) {
        const int row = range_cell(f0, threadIdx.x % ng, nf), part = threadIdx.x / ng;
        if (part < parts) {
          // the columns j = part (mod parts) of the row in increasing order
          T acc = T(0);
#pragma unroll 8
          for (int j = part; j < wrapped; j += parts) acc += ainv[(size_t)j * nf + row] * xc[j];
          const int j0 = f0 + ((part - f0) % parts + parts) % parts;
#pragma unroll 8
          for (int j = j0; j < f1; j += parts) acc += ainv[(size_t)j * nf + row] * xc[j];
          psum[part * nf + row] = acc;
        }
      }
      __syncthreads();
      for (int i = threadIdx.x; i < ng; i += SMALL_BLOCK) {
        const int row = range_cell(f0, i, nf);
        T v = psum[row];
        for (int p = 1; p < parts; ++p) v += psum[p * nf + row];
        e[S.fcell[row]] = v;
      }
      __syncthreads();
    } else {
      small_smooth<T>(S, k, S.coarse_sweeps, lds, sm, first(k), count(k));
    }
  }
  // up: prolong, smooth
  for (int k = S.nlev - 2; k >= 0; --k) {
    const MgTransfer &tr = S.tr[k + 1];
    const T *ec = lds + S.off_e[k + 1];
    T *ef = lds + S.off_e[k];
    const uint32_t *mf = sm + S.off_m[k];
    const uint32_t *mc = sm + S.off_m[k + 1];
    for (int i = threadIdx.x; i < count(k); i += SMALL_BLOCK) {
      const int r = range_cell(first(k), i, tr.f.n);
      if (mf[r] & SOLID_BIT) continue;
      const T e0 = ef[r];
      ef[r] = e0 + prolong_value<T>(tr, r, mc, ec);
    }
    __syncthreads();
    small_smooth<T>(S, k, S.nu2, lds, sm, first(k), count(k));
  }
  for (int i = threadIdx.x; i < count(0); i += SMALL_BLOCK) {
    const int r = range_cell(first(0), i, S.lv[0].n);
    e_out[r] = lds[S.off_e[0] + r];
  }
}

// ---- phi += e --------------------------------------------------------------

template <class T>
__global__ __launch_bounds__(BLOCK) void k_correct(int n, const uint32_t *__restrict__ mask,
                                                   const T *__restrict__ e,
                                                   double *__restrict__ phi,
                                                   const SolveCtl *__restrict__ ctl) {
  if (ctl->done) return;
  const int r = blockIdx.x * BLOCK + threadIdx.x;
  if (r >= n) return;
  if (mask[r] & SOLID_BIT) return;
  phi[r] += double(e[r]);
}

}  // namespace

template <class T>
hipError_t launch_mg_outer_resid(hipStream_t s, const MgLevel &lv, const uint32_t *mask,
                                 const double *src, const double *phi, T *r0, T *e0,
                                 double *partial, SolveCtl *ctl, int add, double *r64,
                                 KrylovCtl *kc, double jacobi, int ring) {
  const int zrun = ring_zrun(lv, ring);
  const int nb = zrun ? ring_blocks(lv, zrun) : (int)blocks_for(lv.n);
  if (zrun)
    hipLaunchKernelGGL(k_outer_resid_ring<T>, dim3(nb), dim3(BLOCK), 0, s, lv, mask, src, phi, r0,
                       e0, partial, ctl, r64, kc, T(jacobi), zrun);
  else
    hipLaunchKernelGGL(k_outer_resid<T>, dim3(nb), dim3(BLOCK), 0, s, lv, mask, src, phi, r0, e0,
                       partial, ctl, r64, kc, T(jacobi));
  hipLaunchKernelGGL(k_final_resid, dim3(1), dim3(FINAL), 0, s, partial, nb, ctl, add);
  return hipGetLastError();
}

template <class T>
hipError_t launch_fcg_apply(hipStream_t s, const MgLevel &lv, const uint32_t *mask, const T *z,
                            const T *q_prev, const T *p_prev, const double *r,
                            double *az, double *partial, KrylovCtl *kc, const SolveCtl *ctl,
                            int ring) {
  const int zrun = ring_zrun(lv, ring);
  const int nb = zrun ? ring_blocks(lv, zrun) : (int)blocks_for(lv.n);
  if (zrun)
    hipLaunchKernelGGL(k_fcg_az_ring<T>, dim3(nb), dim3(BLOCK), 0, s, lv, mask, z, q_prev, p_prev,
                       r, az, partial, ctl, zrun);
  else
    hipLaunchKernelGGL(k_fcg_az<T>, dim3(nb), dim3(BLOCK), 0, s, lv, mask, z, q_prev, p_prev, r,
                       az, partial, ctl);
  hipLaunchKernelGGL(k_fcg_coef, dim3(1), dim3(FINAL), 0, s, partial, nb, kc, ctl);
  return hipGetLastError();
}

template <class T>
hipError_t launch_fcg_update(hipStream_t s, int n, const uint32_t *mask, const T *z,
                             const double *az, T *p, T *q, double *phi, double *r,
                             T *r0, T *e0, double *partial, const KrylovCtl *kc, SolveCtl *ctl,
                             int add, const MgLevel &lv, double jac) {
  const int nb = (int)blocks_for(n);
  hipLaunchKernelGGL(k_fcg_update<T>, dim3(nb), dim3(BLOCK), 0, s, n, mask, z, az, p, q, phi, r,
                     r0, e0, partial, kc, ctl, lv, T(jac), T(lv.h2 / 6.0));
  hipLaunchKernelGGL(k_final_resid, dim3(1), dim3(FINAL), 0, s, partial, nb, ctl, add);
  return hipGetLastError();
}

template <class T>
hipError_t launch_mg_smooth(hipStream_t s, const MgLevel &lv, double omega, int colour,
                            const uint32_t *mask, const T *rhs, T *e, const SolveCtl *ctl) {
  const int hx = (lv.nx + 1) / 2, hy = (lv.ny + 1) / 2;
  hipLaunchKernelGGL(k_smooth<T>, dim3(blocks_for((long)hx * hy * lv.nz)), dim3(BLOCK), 0, s, lv,
                     T(omega), colour, hx, hy, mask, rhs, e, ctl);
  return hipGetLastError();
}

template <class T>
hipError_t launch_jacobi(hipStream_t s, const MgLevel &lv, double omega, double hs,
                         const uint32_t *mask, const T *rhs, const T *x_in, T *x_out,
                         const SolveCtl *ctl, double *phi_add, int ring) {
  const int zrun = ring_zrun(lv, ring);
  if (zrun) {
    const int nb = ring_blocks(lv, zrun);
    if (phi_add)
      hipLaunchKernelGGL((k_jacobi_ring<T, true>), dim3(nb), dim3(BLOCK), 0, s, lv, T(omega),
                         T(hs), mask, rhs, x_in, x_out, ctl, phi_add, zrun);
    else
      hipLaunchKernelGGL((k_jacobi_ring<T, false>), dim3(nb), dim3(BLOCK), 0, s, lv, T(omega),
                         T(hs), mask, rhs, x_in, x_out, ctl, phi_add, zrun);
    return hipGetLastError();
  }
  if (phi_add)
    hipLaunchKernelGGL((k_jacobi<T, true>), dim3(blocks_for(lv.n)), dim3(BLOCK), 0, s, lv,
                       T(omega), T(hs), mask, rhs, x_in, x_out, ctl, phi_add);
  else
    hipLaunchKernelGGL((k_jacobi<T, false>), dim3(blocks_for(lv.n)), dim3(BLOCK), 0, s, lv,
                       T(omega), T(hs), mask, rhs, x_in, x_out, ctl, phi_add);
  return hipGetLastError();
}

template <class T>
hipError_t launch_mg_restrict(hipStream_t s, const MgTransfer &tr, const uint32_t *mf,
                              const uint32_t *mc, const T *rf, const T *ef, T *rc, T *ec,
                              const SolveCtl *ctl, bool tiled, double jac, double hs, int ring) {
  const int zrun = ring_zrun_restrict(tr.f, ring);
  if (zrun) {
    hipLaunchKernelGGL(k_restrict_ring<T>, dim3(ring_blocks(tr.f, zrun)), dim3(BLOCK), 0, s, tr,
                       mf, mc, rf, ef, rc, ec, ctl, T(jac), T(hs), zrun);
    return hipGetLastError();
  }
  // the tiled form where a level is wide enough to fill its tiles (and its
  // planes fit the grid's z extent)
  if (tiled && tr.c.nx >= RT_X && tr.c.ny >= RT_Y && tr.c.nz <= 65535) {
    const dim3 grid((tr.c.nx + RT_X - 1) / RT_X, (tr.c.ny + RT_Y - 1) / RT_Y, tr.c.nz);
    hipLaunchKernelGGL(k_restrict_tiled<T>, grid, dim3(BLOCK), 0, s, tr, mf, mc, rf, ef, rc, ec,
                       ctl, T(jac), T(hs));
  } else {
    hipLaunchKernelGGL(k_restrict<T>, dim3(blocks_for(8L * tr.c.n)), dim3(BLOCK), 0, s, tr, mf,
                       mc, rf, ef, rc, ec, ctl, T(jac), T(hs));
  }
  return hipGetLastError();
}

template <class T>
hipError_t launch_mg_prolong(hipStream_t s, const MgTransfer &tr, const uint32_t *mf,
                             const uint32_t *mc, const T *ec, T *ef, const SolveCtl *ctl,
                             int ring) {
  const int zrun = ring_zrun_restrict(tr.f, ring);
  if (zrun && zrun <= RING_PROLONG_ZRUN) {
    hipLaunchKernelGGL(k_prolong_ring<T>, dim3(ring_blocks(tr.f, zrun)), dim3(BLOCK), 0, s, tr,
                       mf, mc, ec, ef, ctl, zrun);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_prolong<T>, dim3(blocks_for(tr.f.n)), dim3(BLOCK), 0, s, tr, mf, mc, ec,
                     ef, ctl);
  return hipGetLastError();
}

template <class T>
hipError_t launch_mg_coarse(hipStream_t s, const MgLevel &lv, double omega, double jacobi,
                            int sweeps, const uint32_t *mask, const T *rhs, T *e, T *e2,
                            const SolveCtl *ctl) {
  hipLaunchKernelGGL(k_coarse<T>, dim3(1), dim3(COARSE_BLOCK), 0, s, lv, T(omega), T(jacobi),
                     sweeps, mask, rhs, e, e2, ctl);
  return hipGetLastError();
}

template <class T>
hipError_t launch_mg_coarse_dense(hipStream_t s, int nf, const T *ainv, const int *fcell,
                                  const T *rhs, T *e, const SolveCtl *ctl) {
  hipLaunchKernelGGL(k_coarse_dense<T>, dim3(blocks_for(nf)), dim3(BLOCK), 0, s, nf, ainv,
                     fcell, rhs, e, ctl);
  return hipGetLastError();
}

template <class T>
hipError_t prepare_mg_small(size_t lds_bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_mg_small<T>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
}

template <class T>
hipError_t launch_mg_small(hipStream_t s, const MgSmall &S, size_t lds_bytes, const T *r_in,
                           T *e_out, const SolveCtl *ctl) {
  hipLaunchKernelGGL(k_mg_small<T>, dim3(S.ngroups), dim3(SMALL_BLOCK), lds_bytes, s, S, r_in,
                     e_out, ctl);
  return hipGetLastError();
}

template <class T>
hipError_t launch_mg_correct(hipStream_t s, int n, const uint32_t *mask, const T *e, double *phi,
                             const SolveCtl *ctl) {
  hipLaunchKernelGGL(k_correct<T>, dim3(blocks_for(n)), dim3(BLOCK), 0, s, n, mask, e, phi, ctl);
  return hipGetLastError();
}

#define LBE_MG_INSTANTIATE(T)                                                                   \
  template hipError_t launch_mg_outer_resid<T>(hipStream_t, const MgLevel &, const uint32_t *,  \
                                               const double *, const double *, T *, T *,       \
                                               double *, SolveCtl *, int, double *,            \
                                               KrylovCtl *, double, int);                     \
  template hipError_t launch_fcg_apply<T>(hipStream_t, const MgLevel &, const uint32_t *,      \
                                          const T *, const T *, const T *,                      \
                                          const double *, double *, double *, KrylovCtl *,      \
                                          const SolveCtl *, int);                               \
  template hipError_t launch_fcg_update<T>(hipStream_t, int, const uint32_t *, const T *,       \
                                           const double *, T *, T *, double *,                  \
                                           double *, T *, T *, double *, const KrylovCtl *,     \
                                           SolveCtl *, int, const MgLevel &, double);           \
  template hipError_t launch_mg_smooth<T>(hipStream_t, const MgLevel &, double, int,            \
                                          const uint32_t *, const T *, T *, const SolveCtl *);  \
  template hipError_t launch_jacobi<T>(hipStream_t, const MgLevel &, double, double,             \
                                         const uint32_t *, const T *, const T *, T *,           \
                                         const SolveCtl *, double *, int);                      \
  template hipError_t launch_mg_restrict<T>(hipStream_t, const MgTransfer &, const uint32_t *,  \
                                            const uint32_t *, const T *, const T *, T *, T *,   \
                                            const SolveCtl *, bool, double, double, int);       \
  template hipError_t launch_mg_prolong<T>(hipStream_t, const MgTransfer &, const uint32_t *,   \
                                           const uint32_t *, const T *, T *, const SolveCtl *,  \
                                           int);                                                \
  template hipError_t launch_mg_coarse<T>(hipStream_t, const MgLevel &, double, double, int,    \
                                          const uint32_t *, const T *, T *, T *,                \
                                          const SolveCtl *);                                    \
  template hipError_t launch_mg_correct<T>(hipStream_t, int, const uint32_t *, const T *,       \
                                           double *, const SolveCtl *);                         \
  template hipError_t launch_mg_coarse_dense<T>(hipStream_t, int, const T *, const int *,       \
                                                const T *, T *, const SolveCtl *);              \
  template hipError_t prepare_mg_small<T>(size_t);                                              \
  template hipError_t launch_mg_small<T>(hipStream_t, const MgSmall &, size_t, const T *, T *,  \
                                         const SolveCtl *);

LBE_MG_INSTANTIATE(double)
LBE_MG_INSTANTIATE(float)

}  // namespace lbe
