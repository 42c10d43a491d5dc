// lbe_kernels.hip -- HIP kernels (gfx950) of one Lattice Boltzmann
// Electrokinetics time step with metallic electrodes (arXiv:1907.04732).
//
// Data layout in HBM: structure of arrays, site r = x + nx*(y + ny*z), one
// array per population / species / component.  Populations are kept in the
// "pull" form: the array holds post-collision values at the node they left,
// and a step gathers f_i(r) from r - c_i (or from the node's own opposite
// population when r - c_i is solid: halfway bounce-back), collides, and
// writes the result back at r.  Every kernel is one thread per site with
// consecutive threads on consecutive x, so each of the 19 population
// streams and each neighbour read is a contiguous, coalesced access.
//
// FP64 kernels.  All reductions are deterministic: block trees followed by a
// fixed-order combination in the last block to finish.
#include <math.h>

#include "lbe_device.h"
#include "lbe_internal.h"

namespace lbe {

const char *const kKernelNames[KK_COUNT] = {
    "fluid", "ions", "sor", "resid", "charge", "totals", "observe", "sor32", "correct",
    "mg_resid", "mg_smooth", "mg_smooth0", "mg_restrict", "mg_prolong", "mg_coarse", "mg_small",
    "fcg_apply", "fcg_update", "adj_fluid", "adj_ions", "adj_fold",
    "adj_seed", "adj_moments", "rewind", "expand_n", "mg_smooth0_phi", "momentum"};

namespace {

// ---- force on the fluid (reading: excess part of the link flux, Eq. 10,
// projected on the node; Eq. 3 force e rho_el (-grad psi + E_app)) ---------

template <int K>
__device__ __forceinline__ void link_force(const Lattice &L, const Phys &P, int r, uint32_t m,
                                           const Offs &o, const double *__restrict__ phi,
                                           const double *__restrict__ n, double ph,
                                           const double (&nr)[K], double &F0, double &F1,
                                           double &F2) {
  const int N = L.n;
  F0 = F1 = F2 = 0.0;
#pragma unroll
  for (int i = 1; i < NQ; ++i) {
    if (solid_link(m, i)) continue;
    const int rn = nbr(o, r, i);
    const double dphi = phi[rn] - ph - P.Ec[i];
    double g = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k)
      g += excess_link(nr[k], n[k * N + rn], P.z[k] * dphi, 0.5 / LEN[i]);
    const double c = 3.0 * WQ[i] * LEN[i] * g;
    if (CX[i]) F0 += CX[i] * c;
    if (CY[i]) F1 += CY[i] * c;
    if (CZ[i]) F2 += CZ[i] * c;
  }
}

// ---- pass A: link fluxes, force, moments, BGK + Guo forcing --------------
// Each fluid link's excess flux g_k (Eq. 10) is evaluated once and used
// twice: projected on the node as the fluid force, and in the
// diffusion-migration flux j_k = D_k/A0 (g_k - (n_k' - n_k)/Delta_i).  Writes
// post-collision f, u, and n*_k = n_k - sum_i j_k (completed by pass B).

// The arithmetic of pass A at a fluid node r, from its own potential ph and
// concentrations nr and its neighbours' (nb.phi(i), nb.n(k, i) at r + c_i):
// post-collision populations fn, velocity and n* = n - sum_i j.
template <int K, bool NT, class NB>
__device__ __forceinline__ void fluid_node_f64(const Lattice &L, const Phys &P, int r, uint32_t m,
                                               const Offs &o, double ph, const double (&nr)[K],
                                               const NB &nb, const double *__restrict__ fin,
                                               double (&fn)[NQ], double &ux, double &uy,
                                               double &uz, double (&nso)[K]) {
  double js[K];
#pragma unroll
  for (int k = 0; k < K; ++k) js[k] = 0.0;
  double F0 = 0.0, F1 = 0.0, F2 = 0.0;
#pragma unroll
  for (int i = 1; i < NQ; ++i) {
    if (solid_link(m, i)) continue;  // no flux into an electrode
    const double dphi = nb.phi(i) - ph - P.Ec[i];
    double S1, C1;
    sinh_coshm1(dphi, S1, C1);
    double g = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double nt = nb.n(k, i);
      double S, C;
      valence_sc(P.z[k], dphi, S1, C1, S, C);
      const double gk = -((nt + nr[k]) * S + (nt - nr[k]) * C) * (0.5 / LEN[i]);
      g += gk;
      js[k] += P.dk[k] * (gk - (nt - nr[k]) / LEN[i]);
    }
    const double c = 3.0 * WQ[i] * LEN[i] * g;
    if (CX[i]) F0 += CX[i] * c;
    if (CY[i]) F1 += CY[i] * c;
    if (CZ[i]) F2 += CZ[i] * c;
  }

  double f[NQ];
  pull<NT>(L, r, m, o, fin, f);
  double rho = 0.0, m0 = 0.0, m1 = 0.0, m2 = 0.0;
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    rho += f[i];
    if (CX[i]) m0 += CX[i] * f[i];
    if (CY[i]) m1 += CY[i] * f[i];
    if (CZ[i]) m2 += CZ[i] * f[i];
  }
  // Guo forcing: velocity with the half-force shift
  ux = (m0 + 0.5 * F0) / rho;
  uy = (m1 + 0.5 * F1) / rho;
  uz = (m2 + 0.5 * F2) / rho;
  const double uu = ux * ux + uy * uy + uz * uz;
  const double itau = 1.0 / P.tau;
  const double guo = 1.0 - 0.5 * itau;
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const double cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
    const double feq = WQ[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    const double s = ((3.0 * (CX[i] - ux) + 9.0 * cu * CX[i]) * F0 +
                      (3.0 * (CY[i] - uy) + 9.0 * cu * CY[i]) * F1 +
                      (3.0 * (CZ[i] - uz) + 9.0 * cu * CZ[i]) * F2) *
                     (guo * WQ[i]);
    fn[i] = f[i] - (f[i] - feq) * itau + s;
  }
#pragma unroll
  for (int k = 0; k < K; ++k) nso[k] = nr[k] - js[k];
}

// neighbour values gathered into registers
template <int K>
struct FluidRegs64 {
  double p[NQ], nn[K][NQ];
  __device__ __forceinline__ double phi(int i) const { return p[i]; }
  __device__ __forceinline__ double n(int k, int i) const { return nn[k][i]; }
};

template <int K, int TB, bool NT>
__global__ __launch_bounds__(TB) void k_fluid_f64(Lattice L, Phys P,
                                                     const uint32_t *__restrict__ mask,
                                                     const double *__restrict__ phi,
                                                     const double *__restrict__ n,
                                                     const double *__restrict__ fin,
                                                     double *__restrict__ fout,
                                                     double *__restrict__ u,
                                                     double *__restrict__ nstar) {
  const int r = xcd_block(blockIdx.x, gridDim.x, TB, L.nxy, L.xcd) * TB + threadIdx.x;
  if (r >= L.n) return;
  const int N = L.n;
  const uint32_t m = mask[r];
  // Every node stores all its outputs in the same store instructions, a
  // solid node the zeros its slots hold from the start (they are never
  // read): each store then writes whole cache lines, which costs far less
  // than the part-filled lines of a store from the fluid nodes alone.
  double fn[NQ], nso[K], ux = 0.0, uy = 0.0, uz = 0.0;
#pragma unroll
  for (int i = 0; i < NQ; ++i) fn[i] = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) nso[k] = 0.0;
  if (!(m & SOLID_BIT)) {
    Offs o;
    site_offsets(L, r, o);
    const double ph = phi[r];
    double nr[K];
#pragma unroll
    for (int k = 0; k < K; ++k) nr[k] = n[k * N + r];
    // every neighbour's potential and concentrations first, solid
    // neighbours too (their links are skipped): all 18 (1 + K) gathers are
    // then in flight together rather than one link's at a time
    FluidRegs64<K> nb;
#pragma unroll
    for (int i = 1; i < NQ; ++i) {
      const uint32_t rn = nbr(o, r, i);
      nb.p[i] = ld32(phi, rn);
#pragma unroll
      for (int k = 0; k < K; ++k) nb.nn[k][i] = ld32(sbase(n + k * N), rn);
    }
    fluid_node_f64<K, NT>(L, P, r, m, o, ph, nr, nb, fin, fn, ux, uy, uz, nso);
  }
#pragma unroll
  for (int i = 0; i < NQ; ++i) st_stream<NT>(sbase(fout + i * N), r, fn[i]);
  st_stream<NT>(u, r, ux);
  st_stream<NT>(sbase(u + N), r, uy);
  st_stream<NT>(sbase(u + 2 * N), r, uz);
#pragma unroll
  for (int k = 0; k < K; ++k) st_stream<NT>(sbase(nstar + k * N), r, nso[k]);
}

// ---- pass B: advective link fluxes with the step's velocity, new n and
// Poisson source.  J_k = 3 w_i c_i . (n_k u + n_k' u') on every fluid link;
// n_k(t+1) = n*_k - sum_i J_k, updated in place in nio. -------------------

// The advective flux sums at a fluid node, from its velocity and
// concentrations and its neighbours' (nb.cut(i) = c_i . u(r + c_i),
// nb.n(k, i) = n_k(r + c_i)): J_k = sum over fluid links of
// 3 w_i (n_k c_i . u + n_k' c_i . u').
template <int K, class NB>
__device__ __forceinline__ void ions_flux_f64(uint32_t m, double ux, double uy, double uz,
                                              const double (&nr)[K], const NB &nb,
                                              double (&Js)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) Js[k] = 0.0;
#pragma unroll
  for (int i = 1; i < NQ; ++i) {
    if (solid_link(m, i)) continue;
    double cu_h = 0.0;
    if (CX[i]) cu_h += CX[i] * ux;
    if (CY[i]) cu_h += CY[i] * uy;
    if (CZ[i]) cu_h += CZ[i] * uz;
    const double cu_t = nb.cut(i);
#pragma unroll
    for (int k = 0; k < K; ++k) Js[k] += 3.0 * WQ[i] * (nr[k] * cu_h + nb.n(k, i) * cu_t);
  }
}

// neighbour values gathered into registers
template <int K>
struct IonRegs {
  double c[NQ], nn[K][NQ];
  __device__ __forceinline__ double cut(int i) const { return c[i]; }
  __device__ __forceinline__ double n(int k, int i) const { return nn[k][i]; }
};

template <int K, int TB, bool NT>
__global__ __launch_bounds__(TB) void k_ions_f64(Lattice L, Phys P,
                                                    const uint32_t *__restrict__ mask,
                                                    const double *__restrict__ u,
                                                    const double *__restrict__ n,
                                                    double *__restrict__ nio,
                                                    double *__restrict__ src, int order,
                                                    double *__restrict__ phi,
                                                    double *__restrict__ prev) {
  const int r = xcd_block(blockIdx.x, gridDim.x, TB, L.nxy, L.xcd) * TB + threadIdx.x;
  if (r >= L.n) return;
  const int N = L.n;
  const uint32_t m = mask[r];
  const bool solid = m & SOLID_BIT;
  // all nodes store, as in pass A (a solid node its zeros)
  double no[K], q = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) no[k] = 0.0;
  if (!solid) {
    Offs o;
    site_offsets(L, r, o);
    const double ux = u[r], uy = u[N + r], uz = u[2 * N + r];
    double nr[K], Js[K];
#pragma unroll
    for (int k = 0; k < K; ++k) nr[k] = n[k * N + r];
    // c_i . u and the concentrations at every neighbour, loaded before any
    // is used (solid neighbours too, skipped below)
    IonRegs<K> nb;
#pragma unroll
    for (int i = 1; i < NQ; ++i) {
      const uint32_t rn = nbr(o, r, i);
      double c = 0.0;
      if (CX[i]) c += CX[i] * ld32(u, rn);
      if (CY[i]) c += CY[i] * ld32(sbase(u + N), rn);
      if (CZ[i]) c += CZ[i] * ld32(sbase(u + 2 * N), rn);
      nb.c[i] = c;
#pragma unroll
      for (int k = 0; k < K; ++k) nb.nn[k][i] = ld32(sbase(n + k * N), rn);
    }
    ions_flux_f64<K>(m, ux, uy, uz, nr, nb, Js);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      no[k] = nio[k * N + r] - Js[k];
      q += P.z[k] * no[k];
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) st_stream<NT>(sbase(nio + k * N), r, no[k]);
  st_stream<NT>(src, r, P.src_scale * q);
  if (prev) extrapolate_at(r, N, order, solid, phi, prev);
}

// Pass B on LDS-staged tiles of TILE_X x TILE_Y nodes marching through
// TILE_Z planes, as the mixed form's k_ions_f32_tiled: the velocity and the
// concentrations of the planes z - 1, z, z + 1 (with the x, y halo) in a
// ring of four LDS slots, the plane z + 2 and the node's own flag word and
// n* loading meanwhile, one barrier per plane.  The gathering kernel's
// arithmetic on the same values, hence the same bits.  Five FP64 values
// per halo cell fill 54 KB of LDS for two species, so one or two species.
// neighbour values from the LDS slots of a tile: the plane z + c_z in slot
// (k + c_z) & 3 with k = z - z0 + 1, halo cell hc + c_x + RING_HX c_y
template <int K>
struct IonLds {
  const double (*sv)[3 + K][RING_HP];
  int k, hc;
  __device__ __forceinline__ int slot(int i) const { return (k + CZ[i]) & 3; }
  __device__ __forceinline__ int cell(int i) const { return hc + CX[i] + RING_HX * CY[i]; }
  __device__ __forceinline__ double cut(int i) const {
    double c = 0.0;
    if (CX[i]) c += CX[i] * sv[slot(i)][0][cell(i)];
    if (CY[i]) c += CY[i] * sv[slot(i)][1][cell(i)];
    if (CZ[i]) c += CZ[i] * sv[slot(i)][2][cell(i)];
    return c;
  }
  __device__ __forceinline__ double n(int s, int i) const { return sv[slot(i)][3 + s][cell(i)]; }
};

template <int K, bool NT>
__global__ __launch_bounds__(BLOCK) void k_ions_f64_tiled(Lattice L, Phys P,
                                                         const uint32_t *__restrict__ mask,
                                                         const double *__restrict__ u,
                                                         const double *__restrict__ n,
                                                         double *__restrict__ nio,
                                                         double *__restrict__ src, int order,
                                                         double *__restrict__ phi,
                                                         double *__restrict__ prev) {
  static_assert(K >= 1 && K <= 2, "at most two species in LDS");
  constexpr int NV = 3 + K;
  __shared__ double sv[4][NV][RING_HP];  // [slot][u_x, u_y, u_z, n_0..][halo cell]
  const int N = L.n;
  const RingTile t = ring_tile(L, TILE_Z);
  PlaneRing<double> rv[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) rv[v].init(L, t);
  auto fetch = [&](int z) {
    rv[0].fetch(L, u, z);
    rv[1].fetch(L, sbase(u + N), z);
    rv[2].fetch(L, sbase(u + 2 * N), z);
#pragma unroll
    for (int k = 0; k < K; ++k) rv[3 + k].fetch(L, sbase(n + k * N), z);
  };
  auto put = [&](int slot) {
#pragma unroll
    for (int v = 0; v < NV; ++v) rv[v].put(sv[slot][v]);
  };
  // the plane z0 + k sits in slot (k + 1) & 3
  fetch(t.z0 - 1);
  put(0);
  fetch(t.z0);
  put(1);
  fetch(t.z0 + 1);
  uint32_t rn = t.rxy + (uint32_t)L.nxy * (uint32_t)t.z0;
  uint32_t m_next = ld32(mask, rn);
  double ns_next[K];
#pragma unroll
  for (int k = 0; k < K; ++k) ns_next[k] = ld32(sbase((const double *)nio + k * N), rn);
  for (int z = t.z0; z < t.zend; ++z) {
    const uint32_t r = rn;
    const uint32_t m = m_next;
    double ns[K];
#pragma unroll
    for (int k = 0; k < K; ++k) ns[k] = ns_next[k];
    put((z - t.z0 + 2) & 3);  // plane z + 1
    if (z + 1 < t.zend) {     // in flight during this plane
      fetch(z + 2);
      rn += (uint32_t)L.nxy;
      m_next = ld32(mask, rn);
#pragma unroll
      for (int k = 0; k < K; ++k) ns_next[k] = ld32(sbase((const double *)nio + k * N), rn);
    }
    // the slot just written held plane z - 2, last read in the previous
    // step, which every thread has left at this barrier
    __syncthreads();
    const bool solid = m & SOLID_BIT;
    double no[K], q = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) no[k] = 0.0;
    if (!solid) {
      const int kk = z - t.z0 + 1, s0 = kk & 3;
      const double ux = sv[s0][0][t.hc], uy = sv[s0][1][t.hc], uz = sv[s0][2][t.hc];
      double nr[K], Js[K];
#pragma unroll
      for (int k = 0; k < K; ++k) nr[k] = sv[s0][3 + k][t.hc];
      // the neighbours' values read from LDS link by link
      const IonLds<K> nb{sv, kk, t.hc};
      ions_flux_f64<K>(m, ux, uy, uz, nr, nb, Js);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        no[k] = ns[k] - Js[k];
        q += P.z[k] * no[k];
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) st_stream<NT>(sbase(nio + k * N), r, no[k]);
    st_stream<NT>(src, r, P.src_scale * q);
    if (prev) extrapolate_at((int)r, N, order, solid, phi, prev);
  }
}

// ---- Poisson: one colour of the four-colour SOR sweep (Eqs. 13, 15) --------
// colour(x, y, z) = ((x + z) & 1) + 2 ((y + z) & 1); no two D3Q19 neighbours
// share a colour, so a colour's nodes update independently.

__global__ __launch_bounds__(BLOCK) void k_sor_f64(Lattice L, double omega, int colour, int hx,
                                                   int hy, const uint32_t *__restrict__ mask,
                                                   const double *__restrict__ src,
                                                   double *__restrict__ phi,
                                                   const SolveCtl *__restrict__ ctl) {
  if (ctl->done) return;
  const int t = blockIdx.x * BLOCK + threadIdx.x;
  const int plane = hx * hy;
  if (t >= plane * L.nz) return;
  const int z = t / plane;
  const int rem = t - z * plane;
  const int iy = rem / hx;
  const int ix = rem - iy * hx;
  const int x = 2 * ix + ((colour ^ z) & 1);
  const int y = 2 * iy + (((colour >> 1) ^ z) & 1);
  if (x >= L.nx || y >= L.ny) return;
  const int r = x + L.nx * (y + L.ny * z);
  const uint32_t m = mask[r];
  if (m & SOLID_BIT) return;
  Offs o;
  site_offsets(L, r, o);
  double pn[NQ];
  gather(o, r, phi, pn);
  const double sr = src[r];
  double num = 0.0, den = 0.0;
#pragma unroll
  for (int i = 1; i < NQ; ++i) {
    if ((L.selfm >> (i - 1)) & 1u) continue;
    const double ws = solid_link(m, i) ? L.wall * WQ[i] : WQ[i];
    num += ws * pn[i];
    den += ws;
  }
  num += sr;
  phi[r] = (1.0 - omega) * pn[0] + omega * (num / den);
}

// residual R = L_h phi + 4 pi l_B rho_el = 6 [sum_i w_i s_i (phi' - phi) + src];
// block maxima of |R| into partial[] (second stage: k_final_max)
__global__ __launch_bounds__(BLOCK) void k_resid_f64(Lattice L, const uint32_t *__restrict__ mask,
                                                     const double *__restrict__ src,
                                                     const double *__restrict__ phi,
                                                     double *__restrict__ partial,
                                                     const SolveCtl *__restrict__ ctl) {
  __shared__ double sm[BLOCK / WAVE];
  if (ctl->done) return;
  const int lb = xcd_block(blockIdx.x, gridDim.x, BLOCK, L.nxy, L.xcd);
  const int r = lb * BLOCK + threadIdx.x;
  double a = 0.0;
  if (r < L.n) {
    const uint32_t m = mask[r];
    if (!(m & SOLID_BIT)) {
      Offs o;
      site_offsets(L, r, o);
      double pn[NQ];
      gather(o, r, phi, pn);
      const double sr = src[r];
      double acc = 0.0;
#pragma unroll
      for (int i = 1; i < NQ; ++i) {
        if ((L.selfm >> (i - 1)) & 1u) continue;
        const double ws = solid_link(m, i) ? L.wall * WQ[i] : WQ[i];
        acc += ws * (pn[i] - pn[0]);
      }
      a = fabs(6.0 * (acc + sr));
    }
  }
  a = block_max(a, sm);
  if (threadIdx.x == 0) partial[lb] = a;
}

// ---- electrode charge (Eq. 16): Q_e = -(6/4 pi l_B) sum over the electrode's
// interface nodes of sum_{fluid links} 2 w_i (phi' - phi_s) ----------------

__global__ __launch_bounds__(BLOCK) void k_charge(Lattice L, double q_scale,
                                                  const uint32_t *__restrict__ mask,
                                                  const double *__restrict__ phi,
                                                  const int *__restrict__ iface_site,
                                                  const int *__restrict__ blk_begin,
                                                  const int *__restrict__ blk_end,
                                                  double *__restrict__ partial,
                                                  const SolveCtl *__restrict__ gate) {
  __shared__ double sm[BLOCK / WAVE];
  if (gate && (!gate->done || gate->nonfinite)) return;  // queued ahead of a solve that has not converged
  const int b = blockIdx.x;
  const int idx = blk_begin[b] + threadIdx.x;
  double v = 0.0;
  if (idx < blk_end[b]) {
    const int r = iface_site[idx];
    const uint32_t m = mask[r];
    Offs o;
    site_offsets(L, r, o);
    // only the fluid neighbours' potentials: an interface site has few, and
    // the sites of a wavefront lie scattered over the electrode's surface,
    // so each load touches its own cache lines
    const double p0 = ld32(phi, (uint32_t)r);
    double pn[NQ];
#pragma unroll
    for (int i = 1; i < NQ; ++i)
      if (!solid_link(m, i)) pn[i] = ld32(phi, (uint32_t)nbr(o, r, i));
    double lap = 0.0;
#pragma unroll
    for (int i = 1; i < NQ; ++i) {
      if (solid_link(m, i)) continue;
      lap += WQ[i] * L.wall * (pn[i] - p0);
    }
    v = q_scale * lap;
  }
  v = block_sum(v, sm);
  if (threadIdx.x == 0) partial[b] = v;
}

// Per electrode (one block each), compensated sum of its blocks' partials:
// each thread keeps a Neumaier sum over a strided subset, and the block
// combines the (sum, compensation) pairs in a fixed tree with the exact
// rounding error of every addition carried along.
__device__ __forceinline__ double two_sum_err(double a, double b, double t) {
  return fabs(a) >= fabs(b) ? (a - t) + b : (b - t) + a;
}

__global__ __launch_bounds__(BLOCK) void k_final_charge(const double *__restrict__ partial,
                                                        const int *__restrict__ blk_elec, int nb,
                                                        double *__restrict__ out,
                                                        const SolveCtl *__restrict__ gate) {
  __shared__ double ts[BLOCK], tc[BLOCK];
  if (gate && (!gate->done || gate->nonfinite)) return;
  const int e = blockIdx.x;
  double s = 0.0, c = 0.0;
  for (int k = threadIdx.x; k < nb; k += BLOCK) {
    if (blk_elec[k] != e) continue;
    const double x = partial[k];
    const double t = s + x;
    c += two_sum_err(s, x, t);
    s = t;
  }
  ts[threadIdx.x] = s;
  tc[threadIdx.x] = c;
  __syncthreads();
  for (int h = BLOCK / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      const double a = ts[threadIdx.x], b = ts[threadIdx.x + h], t = a + b;
      tc[threadIdx.x] += tc[threadIdx.x + h] + two_sum_err(a, b, t);
      ts[threadIdx.x] = t;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[e] = ts[0] + tc[0];
}

// ---- conserved totals: mass, ionic charge, species amounts ------------------

__global__ __launch_bounds__(BLOCK) void k_totals_f64(Lattice L, int K, int4 zk,
                                                      const uint32_t *__restrict__ mask,
                                                      const double *__restrict__ fin,
                                                      const double *__restrict__ n,
                                                      double *__restrict__ partial) {
  __shared__ double sm[BLOCK / WAVE];
  const int r = blockIdx.x * BLOCK + threadIdx.x;
  const int N = L.n;
  const int nq = 2 + K;
  const int zz[4] = {zk.x, zk.y, zk.z, zk.w};
  const bool fluid = r < N && !(mask[r] & SOLID_BIT);
  for (int q = 0; q < nq; ++q) {
    double v = 0.0;
    if (fluid) {
      if (q == 0) {
        for (int i = 0; i < NQ; ++i) v += fin[i * N + r];
      } else if (q == 1) {
        for (int k = 0; k < K; ++k) v += zz[k] * n[k * N + r];
      } else {
        v = n[(q - 2) * N + r];
      }
    }
    v = block_sum(v, sm);
    if (threadIdx.x == 0) partial[q * gridDim.x + blockIdx.x] = v;
  }
}

// Total fluid momentum sum_r rho(r) u(r) = sum_r (sum_i f_i c_i + F/2) over
// fluid nodes, from the pre-collision populations and the velocity of Guo
// forcing that the observables kernel wrote (its component along an applied
// field is the electro-osmotic flux).
__global__ __launch_bounds__(BLOCK) void k_momentum(Lattice L, const uint32_t *__restrict__ mask,
                                                    const double *__restrict__ fpre,
                                                    const double *__restrict__ u,
                                                    double *__restrict__ partial) {
  __shared__ double sm[BLOCK / WAVE];
  const int r = blockIdx.x * BLOCK + threadIdx.x;
  const int N = L.n;
  const bool fluid = r < N && !(mask[r] & SOLID_BIT);
  double rho = 0.0;
  if (fluid)
    for (int i = 0; i < NQ; ++i) rho += fpre[i * N + r];
  for (int a = 0; a < 3; ++a) {
    double v = fluid ? rho * u[a * N + r] : 0.0;
    v = block_sum(v, sm);
    if (threadIdx.x == 0) partial[a * gridDim.x + blockIdx.x] = v;
  }
}

// ---- observables: pre-collision populations and the Guo velocity ----------

template <int K>
__global__ __launch_bounds__(BLOCK) void k_observe_f64(Lattice L, Phys P,
                                                       const uint32_t *__restrict__ mask,
                                                       const double *__restrict__ phi,
                                                       const double *__restrict__ n,
                                                       const double *__restrict__ fin,
                                                       double *__restrict__ fpre,
                                                       double *__restrict__ u) {
  const int r = blockIdx.x * BLOCK + threadIdx.x;
  if (r >= L.n) return;
  const int N = L.n;
  const uint32_t m = mask[r];
  if (m & SOLID_BIT) {
    for (int i = 0; i < NQ; ++i) fpre[i * N + r] = 0.0;
    u[r] = u[N + r] = u[2 * N + r] = 0.0;
    return;
  }
  Offs o;
  site_offsets(L, r, o);
  const double ph = phi[r];
  double nr[K];
#pragma unroll
  for (int k = 0; k < K; ++k) nr[k] = n[k * N + r];
  double F0, F1, F2;
  link_force<K>(L, P, r, m, o, phi, n, ph, nr, F0, F1, F2);
  double f[NQ];
  pull(L, r, m, o, fin, f);
  double rho = 0.0, m0 = 0.0, m1 = 0.0, m2 = 0.0;
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    fpre[i * N + r] = f[i];
    rho += f[i];
    if (CX[i]) m0 += CX[i] * f[i];
    if (CY[i]) m1 += CY[i] * f[i];
    if (CZ[i]) m2 += CZ[i] * f[i];
  }
  u[r] = (m0 + 0.5 * F0) / rho;
  u[N + r] = (m1 + 0.5 * F1) / rho;
  u[2 * N + r] = (m2 + 0.5 * F2) / rho;
}

// Rewind of a step whose Poisson solve failed: phi(t), kept by pass B, goes
// back into phi (and, under extrapolation, the history moves back by one),
// and the source is recomputed from n(t) exactly as pass B forms it.
template <int K>
__global__ __launch_bounds__(BLOCK) void k_rewind_f64(Lattice L, Phys P,
                                                      const uint32_t *__restrict__ mask,
                                                      const double *__restrict__ n,
                                                      double *__restrict__ src,
                                                      double *__restrict__ phi,
                                                      double *__restrict__ prev, int shift) {
  const int r = blockIdx.x * BLOCK + threadIdx.x;
  if (r >= L.n || (mask[r] & SOLID_BIT)) return;
  const int N = L.n;
  double q = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) q += P.z[k] * n[k * N + r];
  src[r] = P.src_scale * q;
  phi[r] = prev[r];
  if (shift) prev[r] = prev[N + r];
}

// dst[idx[t]] = val[t]: new potentials of the solid nodes
__global__ __launch_bounds__(BLOCK) void k_scatter(int count, const int *__restrict__ idx,
                                                   const double *__restrict__ val,
                                                   double *__restrict__ dst) {
  const int t = blockIdx.x * BLOCK + threadIdx.x;
  if (t < count) dst[idx[t]] = val[t];
}

}  // namespace

// ---- launchers ------------------------------------------------------------

#define LBE_DISPATCH_K(K, CALL)                 \
  switch (K) {                                  \
    case 1: CALL(1); break;                     \
    case 2: CALL(2); break;                     \
    case 3: CALL(3); break;                     \
    default: CALL(4); break;                    \
  }

hipError_t launch_fluid_f64(hipStream_t s, const Lattice &L, const Phys &P, const uint32_t *mask,
                            const double *phi, const double *n, const double *fin, double *fout,
                            double *u, double *nstar, int tb, bool nt) {
#define CALL(KK, TB, NT) \
  hipLaunchKernelGGL((k_fluid_f64<KK, TB, NT>), dim3((L.n + TB - 1) / TB), dim3(TB), 0, s, L, P, mask, phi, n, fin, fout, u, nstar)
  LBE_DISPATCH_K_TB_NT(P.K, tb, nt, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_ions_f64(hipStream_t s, const Lattice &L, const Phys &P, const uint32_t *mask,
                           const double *u, const double *n, double *nio, double *src, int order,
                           double *phi, double *prev, int tb, bool nt) {
  if (tb == TB_TILED) {
    if (!tiles_fit(L) || P.K > 2) return hipErrorInvalidValue;
    const unsigned nb = (unsigned)((L.nx / TILE_X) * (L.ny / TILE_Y) *
                                   ((L.nz + TILE_Z - 1) / TILE_Z));
#define CALL(KK, NT) \
  hipLaunchKernelGGL((k_ions_f64_tiled<KK, NT>), dim3(nb), dim3(BLOCK), 0, s, L, P, mask, u, n, nio, src, order, phi, prev)
    if (P.K == 1) {
      if (nt) CALL(1, true); else CALL(1, false);
    } else {
      if (nt) CALL(2, true); else CALL(2, false);
    }
#undef CALL
    return hipGetLastError();
  }
#define CALL(KK, TB, NT) \
  hipLaunchKernelGGL((k_ions_f64<KK, TB, NT>), dim3((L.n + TB - 1) / TB), dim3(TB), 0, s, L, P, mask, u, n, nio, src, order, phi, prev)
  LBE_DISPATCH_K_TB_NT(P.K, tb, nt, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_rewind_f64(hipStream_t s, const Lattice &L, const Phys &P, const uint32_t *mask,
                             const double *n, double *src, double *phi, double *prev, int shift) {
#define CALL(KK) \
  hipLaunchKernelGGL(k_rewind_f64<KK>, dim3(blocks_for(L.n)), dim3(BLOCK), 0, s, L, P, mask, n, src, phi, prev, shift)
  LBE_DISPATCH_K(P.K, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_sor_f64(hipStream_t s, const Lattice &L, const Phys &P, int colour,
                          const uint32_t *mask, const double *src, double *phi,
                          const SolveCtl *ctl) {
  const int hx = (L.nx + 1) / 2, hy = (L.ny + 1) / 2;
  const long threads = (long)hx * hy * L.nz;
  hipLaunchKernelGGL(k_sor_f64, dim3(blocks_for(threads)), dim3(BLOCK), 0, s, L, P.omega, colour,
                     hx, hy, mask, src, phi, ctl);
  return hipGetLastError();
}

hipError_t launch_scatter(hipStream_t s, int count, const int *idx, const double *val,
                          double *dst) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter, dim3(blocks_for(count)), dim3(BLOCK), 0, s, count, idx, val, dst);
  return hipGetLastError();
}

int residual_blocks(const Lattice &L) { return (int)blocks_for(L.n); }
int totals_blocks(const Lattice &L) { return (int)blocks_for(L.n); }

hipError_t launch_resid_f64(hipStream_t s, const Lattice &L, const uint32_t *mask,
                            const double *src, const double *phi, double *partial, SolveCtl *ctl,
                            int add) {
  const int nb = (int)blocks_for(L.n);
  hipLaunchKernelGGL(k_resid_f64, dim3(nb), dim3(BLOCK), 0, s, L, mask, src, phi, partial, ctl);
  hipLaunchKernelGGL(k_final_resid, dim3(1), dim3(FINAL), 0, s, partial, nb, ctl, add);
  return hipGetLastError();
}

__global__ void k_ctl_reset(SolveCtl *__restrict__ ctl, double tol) {
  if (threadIdx.x == 0) *ctl = SolveCtl{0.0, tol, 0, 0, 0, 0, 0, 0, 0ull, nullptr};
}

__global__ void k_chunk_status(const SolveCtl *__restrict__ ctl, ChunkStatus *__restrict__ st) {
  if (threadIdx.x != 0) return;
  // a non-finite residual also ends the solve, so done covers both outcomes
  if (!ctl->done) st->unconverged += 1;
  if (ctl->nonfinite) st->nonfinite += 1;
  st->iters += ctl->done ? ctl->iters : ctl->count;
  if (!(ctl->resid <= st->resid_max)) st->resid_max = ctl->resid;
}

hipError_t launch_ctl_reset(hipStream_t s, SolveCtl *ctl, double tol) {
  hipLaunchKernelGGL(k_ctl_reset, dim3(1), dim3(64), 0, s, ctl, tol);
  return hipGetLastError();
}

hipError_t launch_chunk_status(hipStream_t s, const SolveCtl *ctl, ChunkStatus *st) {
  hipLaunchKernelGGL(k_chunk_status, dim3(1), dim3(64), 0, s, ctl, st);
  return hipGetLastError();
}

hipError_t launch_charge(hipStream_t s, const Lattice &L, double q_scale, const uint32_t *mask,
                         const double *phi, const int *iface_site, const int *blk_elec,
                         const int *blk_begin, const int *blk_end, int nblocks, int ne,
                         double *partial, double *out, const SolveCtl *gate) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_charge, dim3(nblocks), dim3(BLOCK), 0, s, L, q_scale, mask, phi,
                     iface_site, blk_begin, blk_end, partial, gate);
  hipLaunchKernelGGL(k_final_charge, dim3(ne), dim3(BLOCK), 0, s, partial, blk_elec, nblocks,
                     out, gate);
  return hipGetLastError();
}

hipError_t launch_totals_f64(hipStream_t s, const Lattice &L, int K, const int *z,
                             const uint32_t *mask, const double *fin, const double *n,
                             double *partial, double *out) {
  int4 zk = make_int4(z[0], K > 1 ? z[1] : 0, K > 2 ? z[2] : 0, K > 3 ? z[3] : 0);
  const int nb = (int)blocks_for(L.n);
  hipLaunchKernelGGL(k_totals_f64, dim3(nb), dim3(BLOCK), 0, s, L, K, zk, mask, fin, n, partial);
  hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(FINAL), 0, s, partial, nb, 2 + K, out);
  return hipGetLastError();
}

hipError_t launch_momentum(hipStream_t s, const Lattice &L, const uint32_t *mask,
                           const double *fpre, const double *u, double *partial, double *out) {
  const int nb = (int)blocks_for(L.n);
  hipLaunchKernelGGL(k_momentum, dim3(nb), dim3(BLOCK), 0, s, L, mask, fpre, u, partial);
  hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(FINAL), 0, s, partial, nb, 3, out);
  return hipGetLastError();
}

hipError_t launch_observe_f64(hipStream_t s, const Lattice &L, const Phys &P,
                              const uint32_t *mask, const double *phi, const double *n,
                              const double *fin, double *fpre, double *u) {
#define CALL(KK) \
  hipLaunchKernelGGL(k_observe_f64<KK>, dim3(blocks_for(L.n)), dim3(BLOCK), 0, s, L, P, mask, phi, n, fin, fpre, u)
  LBE_DISPATCH_K(P.K, CALL)
#undef CALL
  return hipGetLastError();
}

}  // namespace lbe
