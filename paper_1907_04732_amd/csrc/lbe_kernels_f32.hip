// lbe_kernels_f32.hip -- the mixed-precision form of the LBE step (gfx950).
//
// Populations are stored and collided in FP32 as deviations from the rest
// state, h_i = f_i - w_i rho0, and concentrations as deviations from a
// reference, nu_k = n_k - n_ref,k: the physical signals (|u| ~ 1e-4, charge
// densities ~ 1e-3 n_ref) then keep FP32's relative precision instead of
// being rounded against the O(1) background.  Each deviation is held as an
// unevaluated FP32 pair nu = hi + lo (|lo| <= ulp(hi) / 2): the fluxes read hi
// only, and a node's own update adds its increment to the pair with an exact
// two-sum.  A single FP32 word loses every increment below half an ulp of
// the value it is added to; at the large deviations inside a double layer
// that loss is one-signed over thousands of steps, and the ion counts (hence
// the electrode charges) drift.  The pair keeps the update to ~2^-48.  The potential stays FP64: it is
// read once per step, and the differences phi' - phi that drive migration
// (~1e-3 of phi) are taken in FP64 before rounding.  The Poisson source
// (4 pi l_B / 6) rho_el is accumulated in FP64 from the FP32 deviations.
// Same layout and pull-form streaming as the FP64 kernels (lbe_kernels.hip).
#include <math.h>

#include "lbe_device.h"
#include "lbe_internal.h"

namespace lbe {
namespace {

template <int K>
__device__ __forceinline__ void link_force_f32(const Lattice &L, const Phys &P, int r, uint32_t m,
                                               const Offs &o, const double *__restrict__ phi,
                                               const float *__restrict__ nu, double ph,
                                               const float *ref, const float (&nr)[K], float &F0,
                                               float &F1, float &F2) {
  const int N = L.n;
  F0 = F1 = F2 = 0.f;
#pragma unroll
  for (int i = 1; i < NQ; ++i) {
    if (solid_link(m, i)) continue;
    const int rn = nbr(o, r, i);
    const double dphi = phi[rn] - ph - P.Ec[i];
    float g = 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k)
      g += excess_link_f(nr[k], ref[k] + nu[k * N + rn], float(P.z[k] * dphi),
                         float(0.5 / LEN[i]));
    const float c = float(3.0 * WQ[i] * LEN[i]) * g;
    if (CX[i]) F0 += CX[i] * c;
    if (CY[i]) F1 += CY[i] * c;
    if (CZ[i]) F2 += CZ[i] * c;
  }
}

// the source slot is selected, not the load, so all 19 loads are
// unconditional
template <bool NT = false>
__device__ __forceinline__ void pull_f32(const Lattice &L, int r, uint32_t m, const Offs &o,
                                         const float *__restrict__ hin, float (&h)[NQ]) {
  const int N = L.n;
  h[0] = ld_stream<NT>(&hin[r]);
#pragma unroll
  for (int i = 1; i < NQ; ++i) {
    const int j = OPP[i];
    h[i] = ld_stream<NT>(&hin[solid_link(m, j) ? j * N + r : i * N + nbr(o, r, j)]);
  }
}

// Pass A: each fluid link's excess flux (Eq. 10) evaluated once, used for the
// fluid force and for the diffusion-migration flux; collision; writes h, u and
// the increment dnu_k = -sum_i j_k (applied by k_ions_f32).
//
// The arithmetic at a fluid node r, its neighbours' potential and deviations
// taken from nb (nb.phi(i), nb.nu(k, i) at r + c_i).  Writes the new
// populations hn, the velocity and the increments dno.  (Pass A keeps its
// neighbour loads in registers: on LDS tiles like pass B's its population
// pulls cross the tile boundaries at other times than the neighbouring
// tiles read the same lines, which measured 1.06 GB fetched per launch at
// 192^3 against 0.64 GB, for no gain in time.)
template <int K, bool NT, class NB>
__device__ __forceinline__ void fluid_node_f32(const Lattice &L, const Phys &P, int r, uint32_t m,
                                               const Offs &o, double ph, const float (&dv)[K],
                                               const NB &nb, const float *__restrict__ hin,
                                               float (&hn)[NQ], float &ux, float &uy, float &uz,
                                               float (&dno)[K]) {
  // deviation reference of this node's system (fluid neighbours share it),
  // held in registers: the link loop adds it at every neighbour
  const float *refp = P.nref_f + 4 * system_of(m);
  float ref[K], nr[K], js[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    ref[k] = refp[k];
    nr[k] = ref[k] + dv[k];
    js[k] = 0.f;
  }
  // the populations first, so that their loads overlap the link arithmetic
  float h[NQ];
  pull_f32<NT>(L, r, m, o, hin, h);
  // Each link's potential difference in FP64, rounded once.  When every
  // species has |z| = 1 and every fluid link of the wave has |delta| <=
  // 1/8 (a wave-wide vote), the links run without a branch, on the series
  // through delta^5 (sinh) and delta^6 (cosh - 1), whose next terms are
  // below 1e-9 relative there, with a wall link's factors zeroed (no flux
  // into an electrode).  Otherwise the loop below takes each link's own
  // path.
  float dl[NQ];
  float dmax = 0.f;
#pragma unroll
  for (int i = 1; i < NQ; ++i) {
    dl[i] = solid_link(m, i) ? 0.f : float(nb.phi(i) - ph - P.Ec[i]);
    dmax = fmaxf(dmax, fabsf(dl[i]));
  }
  const bool fast = P.unit_z && __all(dmax <= 0.125f);
  float F0 = 0.f, F1 = 0.f, F2 = 0.f;
  if (fast) {
    // per species: n' + n = dnu' + (2 ref + nu) and n' - n = dnu' - nu
    float zf[K], sum0[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      zf[k] = float(P.z[k]);
      sum0[k] = ref[k] + nr[k];
    }
#pragma unroll
    for (int i = 1; i < NQ; ++i) {
      const float open = solid_link(m, i) ? 0.f : 1.f;
      const float d = dl[i], x = d * d;
      // -(sinh, cosh - 1) / (2 |c_i|), and 1 / |c_i|, zero on a wall link
      const float hl = open * float(-0.5 / LEN[i]);
      const float a = hl * (d * (1.f + x * (1.f / 6 + x * (1.f / 120))));
      const float b = hl * (x * (0.5f + x * (1.f / 24 + x * (1.f / 720))));
      const float il = open * float(1.0 / LEN[i]);
      float g = 0.f;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const float dn = nb.nu(k, i);
        const float t = dn - dv[k];
        const float gk = (dn + sum0[k]) * (zf[k] * a) + t * b;
        g += gk;
        // the ideal part uses the deviations directly: (n' - n) = (nu' - nu)
        js[k] += P.dk_f[k] * (gk - t * il);
      }
      const float c = float(3.0 * WQ[i] * LEN[i]) * g;
      if (CX[i]) F0 += CX[i] * c;
      if (CY[i]) F1 += CY[i] * c;
      if (CZ[i]) F2 += CZ[i] * c;
    }
  } else {
#pragma unroll
    for (int i = 1; i < NQ; ++i) {
      if (solid_link(m, i)) continue;  // no flux into an electrode
      const double dphi = nb.phi(i) - ph - P.Ec[i];
      const float d1 = dl[i];
      float S1, C1;
      sinh_coshm1f(d1, S1, C1);
      const float il = float(1.0 / LEN[i]);
      float g = 0.f;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const float dn = nb.nu(k, i);
        const float nt = ref[k] + dn;
        float S, C;
        valence_scf(P.z[k], dphi, d1, S1, C1, S, C);
        const float gk = -((nt + nr[k]) * S + (nt - nr[k]) * C) * float(0.5 / LEN[i]);
        g += gk;
        js[k] += P.dk_f[k] * (gk - (dn - dv[k]) * il);
      }
      const float c = float(3.0 * WQ[i] * LEN[i]) * g;
      if (CX[i]) F0 += CX[i] * c;
      if (CY[i]) F1 += CY[i] * c;
      if (CZ[i]) F2 += CZ[i] * c;
    }
  }

  float drho = 0.f, m0 = 0.f, m1 = 0.f, m2 = 0.f;
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    drho += h[i];
    if (CX[i]) m0 += CX[i] * h[i];
    if (CY[i]) m1 += CY[i] * h[i];
    if (CZ[i]) m2 += CZ[i] * h[i];
  }
  // sum_i w_i rho0 c_i = 0, so the momentum is carried by the deviations
  const float rho = P.rho0_f + drho;
  ux = (m0 + 0.5f * F0) / rho;
  uy = (m1 + 0.5f * F1) / rho;
  uz = (m2 + 0.5f * F2) / rho;
  const float uu = ux * ux + uy * uy + uz * uz;
  const float itau = P.itau_f;
  const float guo = 1.f - 0.5f * itau;
  // Each velocity on its own: forming the pairs c_i, -c_i from shared even
  // and odd parts (w rho 3 c.u added after the rest) measured 11 us faster
  // at 192^3 but tripled the velocity's difference from the FP64 form over
  // the configured runs (coaxial cell, 30000 steps: 1.1e-4 of max |u|
  // against 3.6e-5).
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const float w = float(WQ[i]);
    const float cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
    // equilibrium minus the rest state w_i rho0
    const float heq = w * (drho + rho * (3.f * cu + 4.5f * cu * cu - 1.5f * uu));
    const float s = ((3.f * (CX[i] - ux) + 9.f * cu * CX[i]) * F0 +
                     (3.f * (CY[i] - uy) + 9.f * cu * CY[i]) * F1 +
                     (3.f * (CZ[i] - uz) + 9.f * cu * CZ[i]) * F2) *
                    (guo * w);
    hn[i] = h[i] - (h[i] - heq) * itau + s;
  }
#pragma unroll
  for (int k = 0; k < K; ++k) dno[k] = -js[k];
}

// neighbour values held in registers
template <int K>
struct NbRegs {
  double p[NQ];
  float n[K][NQ];
  __device__ __forceinline__ double phi(int i) const { return p[i]; }
  __device__ __forceinline__ float nu(int k, int i) const { return n[k][i]; }
};

template <int K, int TB, bool NT>
__global__ __launch_bounds__(TB) void k_fluid_f32(Lattice L, Phys P,
                                                     const uint32_t *__restrict__ mask,
                                                     const double *__restrict__ phi,
                                                     const float *__restrict__ nu,
                                                     const float *__restrict__ hin,
                                                     float *__restrict__ hout,
                                                     float *__restrict__ u,
                                                     float *__restrict__ dnu) {
  const int r = xcd_block(blockIdx.x, gridDim.x, TB, L.nxy, L.xcd) * TB + threadIdx.x;
  if (r >= L.n) return;
  const int N = L.n;
  const uint32_t m = mask[r];
  // Every node stores all its outputs in the same store instructions, a
  // solid node the zeros its slots hold from the start (they are never
  // read): each store then writes whole cache lines, which costs far less
  // than the part-filled lines of a store from the fluid nodes alone.
  float hn[NQ], dno[K], ux = 0.f, uy = 0.f, uz = 0.f;
#pragma unroll
  for (int i = 0; i < NQ; ++i) hn[i] = 0.f;
#pragma unroll
  for (int k = 0; k < K; ++k) dno[k] = 0.f;
  if (!(m & SOLID_BIT)) {
    Offs o;
    site_offsets(L, r, o);
    const double ph = phi[r];
    float dv[K];
#pragma unroll
    for (int k = 0; k < K; ++k) dv[k] = nu[k * N + r];
    // every neighbour's potential and deviations first, solid neighbours
    // too (their links are skipped): all 18 (1 + K) gathers are then in
    // flight together rather than one link's at a time behind a branch
    NbRegs<K> nb;
#pragma unroll
    for (int i = 1; i < NQ; ++i) {
      const uint32_t rn = nbr(o, r, i);
      nb.p[i] = ld32(phi, rn);
#pragma unroll
      for (int k = 0; k < K; ++k) nb.n[k][i] = ld32(sbase(nu + k * N), rn);
    }
    fluid_node_f32<K, NT>(L, P, r, m, o, ph, dv, nb, hin, hn, ux, uy, uz, dno);
  }
#pragma unroll
  for (int i = 0; i < NQ; ++i) st_stream<NT>(sbase(hout + i * N), r, hn[i]);
  st_stream<NT>(u, r, ux);
  st_stream<NT>(sbase(u + N), r, uy);
  st_stream<NT>(sbase(u + 2 * N), r, uz);
#pragma unroll
  for (int k = 0; k < K; ++k) st_stream<NT>(sbase(dnu + k * N), r, dno[k]);
}

// neighbour values from the LDS rings of a tile: the plane z + c_z in slot
// (k + c_z) & 3 with k = z - z0 + 1, halo cell hc + c_x + RING_HX c_y
template <int K>
struct NbRing {
  const double (*sp)[RING_HP];
  const float (*sn)[K][RING_HP];
  int k, hc;
  __device__ __forceinline__ int cell(int i) const { return hc + CX[i] + RING_HX * CY[i]; }
  __device__ __forceinline__ double phi(int i) const { return sp[(k + CZ[i]) & 3][cell(i)]; }
  __device__ __forceinline__ float nu(int s, int i) const { return sn[(k + CZ[i]) & 3][s][cell(i)]; }
};

// Pass A on plane rings: a block of RING_TX x RING_TY nodes marches along z
// through zrun planes with the potential and the deviations of the planes
// z - 1, z, z + 1 (with the x, y halo) in LDS, the plane z + 2 loading into
// registers meanwhile.  Only the population pulls remain gathers from
// memory.  Tiles of a run of planes go to one die in consecutive chunks, so
// the pulls that cross a tile's edge find the lines its neighbours fetched
// in that die's L2.  Same arithmetic as k_fluid_f32, hence the same bits.
template <int K, bool NT>
__global__ __launch_bounds__(BLOCK) void k_fluid_f32_ring(Lattice L, Phys P,
                                                         const uint32_t *__restrict__ mask,
                                                         const double *__restrict__ phi,
                                                         const float *__restrict__ nu,
                                                         const float *__restrict__ hin,
                                                         float *__restrict__ hout,
                                                         float *__restrict__ u,
                                                         float *__restrict__ dnu, int zrun) {
  __shared__ double sp[4][RING_HP];
  __shared__ float sn[4][K][RING_HP];
  const int N = L.n;
  const RingTile t = ring_tile(L, zrun);
  PlaneRing<double> rp;
  PlaneRing<float> rn[K];
  rp.init(L, t);
#pragma unroll
  for (int k = 0; k < K; ++k) rn[k].init(L, t);
  auto fetch = [&](int z) {
    rp.fetch(L, phi, z);
#pragma unroll
    for (int k = 0; k < K; ++k) rn[k].fetch(L, sbase(nu + k * N), z);
  };
  auto put = [&](int slot) {
    rp.put(sp[slot]);
#pragma unroll
    for (int k = 0; k < K; ++k) rn[k].put(sn[slot][k]);
  };
  // the plane z0 + k sits in slot (k + 1) & 3
  fetch(t.z0 - 1);
  put(0);
  fetch(t.z0);
  put(1);
  fetch(t.z0 + 1);
  uint32_t rn_next = t.rxy + (uint32_t)L.nxy * (uint32_t)t.z0;
  uint32_t m_next = ld32(mask, rn_next);
  for (int z = t.z0; z < t.zend; ++z) {
    const uint32_t r = rn_next;
    const uint32_t m = m_next;
    put((z - t.z0 + 2) & 3);  // plane z + 1
    if (z + 1 < t.zend) {     // in flight during this plane
      fetch(z + 2);
      rn_next += (uint32_t)L.nxy;
      m_next = ld32(mask, rn_next);
    }
    // the slot just written held plane z - 2, last read in the previous
    // step, which every thread has left at this barrier
    __syncthreads();
    float hn[NQ], dno[K], ux = 0.f, uy = 0.f, uz = 0.f;
#pragma unroll
    for (int i = 0; i < NQ; ++i) hn[i] = 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) dno[k] = 0.f;
    if (!(m & SOLID_BIT)) {
      Offs o;
      site_offsets(L, (int)r, o);
      const int kk = z - t.z0 + 1;
      const double ph = sp[kk & 3][t.hc];
      float dv[K];
#pragma unroll
      for (int k = 0; k < K; ++k) dv[k] = sn[kk & 3][k][t.hc];
      const NbRing<K> nb{sp, sn, kk, t.hc};
      fluid_node_f32<K, NT>(L, P, (int)r, m, o, ph, dv, nb, hin, hn, ux, uy, uz, dno);
    }
#pragma unroll
    for (int i = 0; i < NQ; ++i) st_stream<NT>(sbase(hout + i * N), r, hn[i]);
    st_stream<NT>(u, r, ux);
    st_stream<NT>(sbase(u + N), r, uy);
    st_stream<NT>(sbase(u + 2 * N), r, uz);
#pragma unroll
    for (int k = 0; k < K; ++k) st_stream<NT>(sbase(dnu + k * N), r, dno[k]);
  }
}

// Pass B: advective link fluxes J_k = 3 w_i c_i . (n_k u + n_k' u') with the
// step's velocity; the step's increment t = dnu_k - sum_i J_k (dnu_k from pass
// A, in nuio) goes onto the pair (nu, lo_in) of nu_k(t): lo + t first (both
// small), then the two-sum of hi with it gives the new pair, hi to nuio and lo
// to lo_out.  Poisson source (4 pi l_B / 6) rho_el accumulated in FP64 from
// hi + lo.
//
// The arithmetic at a fluid node, from its own values (u, the deviations hv,
// the low words lo and pass A's increments dn) and its neighbours' (cut[i] =
// c_i . u(r + c_i), nn[k][i] = nu_k(r + c_i)); returns sum_k z_k n_k.
template <int K>
__device__ __forceinline__ double ions_node_f32(const Phys &P, uint32_t m, float ux, float uy,
                                                float uz, const float (&hv)[K],
                                                const float (&lo)[K], const float (&dn)[K],
                                                const float (&cut)[NQ],
                                                const float (&nn)[K][NQ], float (&hio)[K],
                                                float (&loo)[K]) {
  const int sy = system_of(m);
  const float *ref = P.nref_f + 4 * sy;
  float nr[K], Js[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    nr[k] = ref[k] + hv[k];
    Js[k] = 0.f;
  }
#pragma unroll
  for (int i = 1; i < NQ; ++i) {
    if (solid_link(m, i)) continue;
    float cu_h = 0.f;
    if (CX[i]) cu_h += CX[i] * ux;
    if (CY[i]) cu_h += CY[i] * uy;
    if (CZ[i]) cu_h += CZ[i] * uz;
    const float cu_t = cut[i];
    const float w3 = float(3.0 * WQ[i]);
#pragma unroll
    for (int k = 0; k < K; ++k)
      Js[k] += w3 * (nr[k] * cu_h + (ref[k] + nn[k][i]) * cu_t);
  }
  double q = P.qref[sy];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const float t = lo[k] + (dn[k] - Js[k]);
    two_sum_f(hv[k], t, hio[k], loo[k]);
    q += P.z[k] * (double(hio[k]) + double(loo[k]));
  }
  return q;
}

// c_i . u for a neighbour's velocity components
__device__ __forceinline__ float c_dot(int i, float vx, float vy, float vz) {
  float c = 0.f;
  if (CX[i]) c += CX[i] * vx;
  if (CY[i]) c += CY[i] * vy;
  if (CZ[i]) c += CZ[i] * vz;
  return c;
}

template <int K, int TB, bool NT>
__global__ __launch_bounds__(TB) void k_ions_f32(Lattice L, Phys P,
                                                    const uint32_t *__restrict__ mask,
                                                    const float *__restrict__ u,
                                                    const float *__restrict__ nu,
                                                    const float *__restrict__ lo_in,
                                                    float *__restrict__ nuio,
                                                    float *__restrict__ lo_out,
                                                    double *__restrict__ src, int order,
                                                    double *__restrict__ phi,
                                                    double *__restrict__ prev) {
  const int r = blockIdx.x * TB + threadIdx.x;
  if (r >= L.n) return;
  const int N = L.n;
  const uint32_t m = mask[r];
  const bool solid = m & SOLID_BIT;
  // all nodes store, as in pass A (a solid node its zeros)
  float hio[K], loo[K];
  double q = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) hio[k] = loo[k] = 0.f;
  if (!solid) {
    Offs o;
    site_offsets(L, r, o);
    const float ux = u[r], uy = u[N + r], uz = u[2 * N + r];
    float hv[K], lo[K], dn[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      hv[k] = nu[k * N + r];
      lo[k] = lo_in[k * N + r];
      dn[k] = nuio[k * N + r];
    }
    // c_i . u and the deviations at every neighbour, loaded before any is
    // used (solid neighbours too, skipped by the link loop)
    float cut[NQ], nn[K][NQ];
#pragma unroll
    for (int i = 1; i < NQ; ++i) {
      const uint32_t rn = nbr(o, r, i);
      cut[i] = c_dot(i, CX[i] ? ld32(u, rn) : 0.f, CY[i] ? ld32(sbase(u + N), rn) : 0.f,
                     CZ[i] ? ld32(sbase(u + 2 * N), rn) : 0.f);
#pragma unroll
      for (int k = 0; k < K; ++k) nn[k][i] = ld32(sbase(nu + k * N), rn);
    }
    q = ions_node_f32<K>(P, m, ux, uy, uz, hv, lo, dn, cut, nn, hio, loo);
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    st_stream<NT>(sbase(nuio + k * N), r, hio[k]);
    st_stream<NT>(sbase(lo_out + k * N), r, loo[k]);
  }
  st_stream<NT>(src, r, P.src_scale * q);
  if (prev) extrapolate_at(r, N, order, solid, phi, prev);
}

// Pass B on an LDS-staged tile: a block of TILE_X x TILE_Y nodes (the plane
// rings' tiles) marches along z through TILE_Z planes, keeping the planes
// z - 1, z, z + 1 of the velocity and the deviations (with a one-node halo
// in x and y, wrapped periodically) in LDS, so each value is read from
// memory once per tile instead of once per neighbour.  The plane z + 2 is
// loaded into registers while the plane z is computed and goes to LDS at
// the next step (a ring of four slots), so its latency hides behind the
// arithmetic.  Same arithmetic as k_ions_f32, hence the same bits.  Needs
// nx a multiple of TILE_X and ny of TILE_Y.
template <int K, bool NT>
__global__ __launch_bounds__(BLOCK) void k_ions_f32_tiled(
    Lattice L, Phys P, const uint32_t *__restrict__ mask, const float *__restrict__ u,
    const float *__restrict__ nu, const float *__restrict__ lo_in, float *__restrict__ nuio,
    float *__restrict__ lo_out, double *__restrict__ src, int order,
    double *__restrict__ phi, double *__restrict__ prev) {
  constexpr int NV = 3 + K;
  __shared__ float sv[4][NV][RING_HP];  // [slot][u_x, u_y, u_z, nu_0..][halo cell]
  const int N = L.n;
  const RingTile t = ring_tile(L, TILE_Z);
  PlaneRing<float> rv[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) rv[v].init(L, t);
  auto fetch = [&](int z) {
    rv[0].fetch(L, u, z);
    rv[1].fetch(L, sbase(u + N), z);
    rv[2].fetch(L, sbase(u + 2 * N), z);
#pragma unroll
    for (int k = 0; k < K; ++k) rv[3 + k].fetch(L, sbase(nu + k * N), z);
  };
  auto put = [&](int slot) {
#pragma unroll
    for (int v = 0; v < NV; ++v) rv[v].put(sv[slot][v]);
  };
  const int z0 = t.z0, zend = t.zend, hc = t.hc;
  // the plane z sits in slot (z - z0 + 1) & 3
  fetch(z0 - 1);
  put(0);
  fetch(z0);
  put(1);
  fetch(z0 + 1);
  // the node's own flag word, low words and pass A increments, one plane
  // ahead as well
  uint32_t m_next;
  float lo_next[K], dn_next[K];
  auto fetch_own = [&](int z) {
    const uint32_t r = t.rxy + (uint32_t)L.nxy * z;
    m_next = ld32(mask, r);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      lo_next[k] = ld32(sbase(lo_in + k * N), r);
      dn_next[k] = ld32(sbase((const float *)nuio + k * N), r);
    }
  };
  fetch_own(z0);
  for (int z = z0; z < zend; ++z) {
    put((z - z0 + 2) & 3);                   // plane z + 1
    const uint32_t m = m_next;
    float lo[K], dn[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      lo[k] = lo_next[k];
      dn[k] = dn_next[k];
    }
    if (z + 1 < zend) {                      // in flight during this plane
      fetch(z + 2);
      fetch_own(z + 1);
    }
    __syncthreads();
    const int r = (int)(t.rxy + (uint32_t)L.nxy * z);
    const bool solid = m & SOLID_BIT;
    float hio[K], loo[K];
    double q = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) hio[k] = loo[k] = 0.f;
    if (!solid) {
      const int s0 = (z - z0 + 1) & 3;
      const float ux = sv[s0][0][hc], uy = sv[s0][1][hc], uz = sv[s0][2][hc];
      float hv[K];
#pragma unroll
      for (int k = 0; k < K; ++k) hv[k] = sv[s0][3 + k][hc];
      float cut[NQ], nn[K][NQ];
#pragma unroll
      for (int i = 1; i < NQ; ++i) {
        const int sl = (z - z0 + 1 + CZ[i]) & 3, cc = hc + CX[i] + RING_HX * CY[i];
        cut[i] = c_dot(i, CX[i] ? sv[sl][0][cc] : 0.f, CY[i] ? sv[sl][1][cc] : 0.f,
                       CZ[i] ? sv[sl][2][cc] : 0.f);
#pragma unroll
        for (int k = 0; k < K; ++k) nn[k][i] = sv[sl][3 + k][cc];
      }
      q = ions_node_f32<K>(P, m, ux, uy, uz, hv, lo, dn, cut, nn, hio, loo);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      st_stream<NT>(sbase(nuio + k * N), r, hio[k]);
      st_stream<NT>(sbase(lo_out + k * N), r, loo[k]);
    }
    st_stream<NT>(src, r, P.src_scale * q);
    if (prev) extrapolate_at(r, N, order, solid, phi, prev);
    // no second barrier: the slot the next step fills held plane z - 2,
    // read in the previous step, which every thread left at this step's
    // barrier
  }
}

template <int K>
__global__ __launch_bounds__(BLOCK) void k_observe_f32(Lattice L, Phys P,
                                                       const uint32_t *__restrict__ mask,
                                                       const double *__restrict__ phi,
                                                       const float *__restrict__ nu,
                                                       const float *__restrict__ hin,
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
  const float *ref = P.nref_f + 4 * system_of(m);
  float nr[K];
#pragma unroll
  for (int k = 0; k < K; ++k) nr[k] = ref[k] + nu[k * N + r];
  float F0, F1, F2;
  link_force_f32<K>(L, P, r, m, o, phi, nu, ph, ref, nr, F0, F1, F2);
  float h[NQ];
  pull_f32(L, r, m, o, hin, h);
  double drho = 0.0, m0 = 0.0, m1 = 0.0, m2 = 0.0;
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    fpre[i * N + r] = WQ[i] * P.rho0_d + double(h[i]);
    drho += h[i];
    if (CX[i]) m0 += CX[i] * double(h[i]);
    if (CY[i]) m1 += CY[i] * double(h[i]);
    if (CZ[i]) m2 += CZ[i] * double(h[i]);
  }
  const double rho = P.rho0_d + drho;
  u[r] = (m0 + 0.5 * F0) / rho;
  u[N + r] = (m1 + 0.5 * F1) / rho;
  u[2 * N + r] = (m2 + 0.5 * F2) / rho;
}

__global__ __launch_bounds__(BLOCK) void k_totals_f32(Lattice L, Phys P,
                                                      const uint32_t *__restrict__ mask,
                                                      const float *__restrict__ hin,
                                                      const float *__restrict__ nu,
                                                      const float *__restrict__ lo,
                                                      double *__restrict__ partial) {
  __shared__ double sm[BLOCK / WAVE];
  const int r = blockIdx.x * BLOCK + threadIdx.x;
  const int N = L.n;
  const int K = P.K;
  const int nq = 2 + K;
  const uint32_t m = r < N ? mask[r] : SOLID_BIT;
  const bool fluid = !(m & SOLID_BIT);
  const double *ref = P.nref_d + 4 * system_of(m);
  for (int q = 0; q < nq; ++q) {
    double v = 0.0;
    if (fluid) {
      if (q == 0) {
        v = P.rho0_d;
        for (int i = 0; i < NQ; ++i) v += double(hin[i * N + r]);
      } else if (q == 1) {
        for (int k = 0; k < K; ++k)
          v += P.z[k] * (ref[k] + (double(nu[k * N + r]) + double(lo[k * N + r])));
      } else {
        v = ref[q - 2] + (double(nu[(q - 2) * N + r]) + double(lo[(q - 2) * N + r]));
      }
    }
    v = block_sum(v, sm);
    if (threadIdx.x == 0) partial[q * gridDim.x + blockIdx.x] = v;
  }
}

// Rewind of a step whose Poisson solve failed (as k_rewind_f64): phi(t) back
// from the copy pass B kept, the source recomputed from the pair nu(t) + lo(t)
// as pass B forms it.
template <int K>
__global__ __launch_bounds__(BLOCK) void k_rewind_f32(Lattice L, Phys P,
                                                      const uint32_t *__restrict__ mask,
                                                      const float *__restrict__ nu,
                                                      const float *__restrict__ lo,
                                                      double *__restrict__ src,
                                                      double *__restrict__ phi,
                                                      double *__restrict__ prev, int shift) {
  const int r = blockIdx.x * BLOCK + threadIdx.x;
  if (r >= L.n) return;
  const uint32_t m = mask[r];
  if (m & SOLID_BIT) return;
  const int N = L.n;
  double q = P.qref[system_of(m)];
#pragma unroll
  for (int k = 0; k < K; ++k) q += P.z[k] * (double(nu[k * N + r]) + double(lo[k * N + r]));
  src[r] = P.src_scale * q;
  phi[r] = prev[r];
  if (shift) prev[r] = prev[N + r];
}

// Concentrations in FP64, n = n_ref + (nu + lo) on fluid nodes and 0 on solid
// ones (species-major, as the host copy of the observables).
__global__ __launch_bounds__(BLOCK) void k_expand_n_f32(Lattice L, int K, const double *__restrict__ nref,
                                                        const uint32_t *__restrict__ mask,
                                                        const float *__restrict__ nu,
                                                        const float *__restrict__ lo,
                                                        double *__restrict__ n) {
  const int r = blockIdx.x * BLOCK + threadIdx.x;
  if (r >= L.n) return;
  const uint32_t m = mask[r];
  const int N = L.n;
  for (int k = 0; k < K; ++k)
    n[k * N + r] = (m & SOLID_BIT) ? 0.0
                                   : nref[4 * system_of(m) + k] +
                                         (double(nu[k * N + r]) + double(lo[k * N + r]));
}

}  // namespace

#define LBE_DISPATCH_K(K, CALL) \
  switch (K) {                  \
    case 1: CALL(1); break;     \
    case 2: CALL(2); break;     \
    case 3: CALL(3); break;     \
    default: CALL(4); break;    \
  }

hipError_t launch_fluid_f32(hipStream_t s, const Lattice &L, const Phys &P, const uint32_t *mask,
                            const double *phi, const float *nu, const float *hin, float *hout,
                            float *u, float *dnu, int tb, bool nt) {
  if (tb == TB_TILED) {
    if (!rings_fit(L)) return hipErrorInvalidValue;
    const int zrun = RING_ZRUN;
    const unsigned nb = (unsigned)((L.nx / RING_TX) * (L.ny / RING_TY) * ((L.nz + zrun - 1) / zrun));
#define CALL(KK, NT) \
  hipLaunchKernelGGL((k_fluid_f32_ring<KK, NT>), dim3(nb), dim3(BLOCK), 0, s, L, P, mask, phi, nu, hin, hout, u, dnu, zrun)
#define CALL_T(KK) CALL(KK, true)
#define CALL_F(KK) CALL(KK, false)
    if (nt) {
      LBE_DISPATCH_K(P.K, CALL_T)
    } else {
      LBE_DISPATCH_K(P.K, CALL_F)
    }
#undef CALL_T
#undef CALL_F
#undef CALL
    return hipGetLastError();
  }
#define CALL(KK, TB, NT) \
  hipLaunchKernelGGL((k_fluid_f32<KK, TB, NT>), dim3((L.n + TB - 1) / TB), dim3(TB), 0, s, L, P, mask, phi, nu, hin, hout, u, dnu)
  LBE_DISPATCH_K_TB_NT(P.K, tb, nt, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_rewind_f32(hipStream_t s, const Lattice &L, const Phys &P, const uint32_t *mask,
                             const float *nu, const float *lo, double *src, double *phi,
                             double *prev, int shift) {
#define CALL(KK) \
  hipLaunchKernelGGL(k_rewind_f32<KK>, dim3(blocks_for(L.n)), dim3(BLOCK), 0, s, L, P, mask, nu, lo, src, phi, prev, shift)
  LBE_DISPATCH_K(P.K, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_expand_n_f32(hipStream_t s, const Lattice &L, const Phys &P,
                               const uint32_t *mask, const float *nu, const float *lo, double *n) {
  hipLaunchKernelGGL(k_expand_n_f32, dim3(blocks_for(L.n)), dim3(BLOCK), 0, s, L, P.K, P.nref_d,
                     mask, nu, lo, n);
  return hipGetLastError();
}

hipError_t launch_ions_f32(hipStream_t s, const Lattice &L, const Phys &P, const uint32_t *mask,
                           const float *u, const float *nu, const float *lo_in, float *nuio,
                           float *lo_out, double *src, int order, double *phi, double *prev,
                           int tb, bool nt) {
  if (tb == TB_TILED) {
    if (!tiles_fit(L)) return hipErrorInvalidValue;
    const unsigned nb = (unsigned)((L.nx / TILE_X) * (L.ny / TILE_Y) *
                                   ((L.nz + TILE_Z - 1) / TILE_Z));
#define CALL(KK, NT) \
  hipLaunchKernelGGL((k_ions_f32_tiled<KK, NT>), dim3(nb), dim3(BLOCK), 0, s, L, P, mask, u, nu, lo_in, nuio, lo_out, src, order, phi, prev)
#define CALL_T(KK) CALL(KK, true)
#define CALL_F(KK) CALL(KK, false)
    if (nt) {
      LBE_DISPATCH_K(P.K, CALL_T)
    } else {
      LBE_DISPATCH_K(P.K, CALL_F)
    }
#undef CALL_T
#undef CALL_F
#undef CALL
    return hipGetLastError();
  }
#define CALL(KK, TB, NT) \
  hipLaunchKernelGGL((k_ions_f32<KK, TB, NT>), dim3((L.n + TB - 1) / TB), dim3(TB), 0, s, L, P, mask, u, nu, lo_in, nuio, lo_out, src, order, phi, prev)
  LBE_DISPATCH_K_TB_NT(P.K, tb, nt, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_observe_f32(hipStream_t s, const Lattice &L, const Phys &P,
                              const uint32_t *mask, const double *phi, const float *nu,
                              const float *hin, double *fpre, double *u) {
#define CALL(KK) \
  hipLaunchKernelGGL(k_observe_f32<KK>, dim3(blocks_for(L.n)), dim3(BLOCK), 0, s, L, P, mask, phi, nu, hin, fpre, u)
  LBE_DISPATCH_K(P.K, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_totals_f32(hipStream_t s, const Lattice &L, const Phys &P, const uint32_t *mask,
                             const float *hin, const float *nu, const float *lo, double *partial,
                             double *out) {
  const int nb = (int)blocks_for(L.n);
  hipLaunchKernelGGL(k_totals_f32, dim3(nb), dim3(BLOCK), 0, s, L, P, mask, hin, nu, lo, partial);
  hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(FINAL), 0, s, partial, nb, 2 + P.K, out);
  return hipGetLastError();
}

}  // namespace lbe
