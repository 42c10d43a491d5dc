// lbe_adjoint.hip -- reverse-mode (adjoint) kernels of the FP64 time step
// (gfx950).  They give the gradient of a weighted sum of electrode charges
// and of the fluid momentum, L = sum_e qbar_e Q_e(T) (Eq. 16) +
// ubar . sum_r rho u(r, T), with respect to the electrode potentials, the
// Bjerrum length and the initial state, by running the step of Secs. II B-C
// backwards.
//
// State at time t: stored (post-collision, pull-form) populations P_t, ion
// concentrations n_t, and phi_t = Phi(n_t), the Poisson solution for n_t.
// The collision depends on the pre-collision populations only through their
// density and momentum, so a recomputed state is kept as (rho, m, n, phi):
// k_adj_moments takes the moments of the pulled populations.  The state may
// be stored in FP64 or in the mixed form (FP32 deviations h = f - w rho0 and
// nu = n - n_ref); the adjoint arithmetic is FP64 either way.
// Adjoint state: A_t = dL/d(pre-collision populations at t) and
// nb_t = dL/dn_t with phi_t's dependence on n_t already folded in.
//
// One reverse step t+1 -> t (the state at t is recomputed from a checkpoint):
//  1. k_adj_fluid: the adjoint of streaming (a gather of A_{t+1} along +c_i,
//     or the node's own opposite slot across a wall), of the BGK collision
//     with the Guo source, and of u = (m + F/2)/rho; the velocity also feeds
//     the advective link fluxes, whose share of the velocity adjoint is
//     gathered here.  Writes A_t, the force adjoint Fb and u.
//  2. k_adj_ions: the adjoint of the link fluxes of Eq. 10 (diffusion,
//     migration, advection) and of the force they exert, per link pair:
//     both ends of a fluid link see the same flux with opposite signs, so the
//     pair's adjoint is  Gb_k = d_k (nb_k(r') - nb_k(r)) + 3 w_i Delta_i
//     c_i . (Fb(r) + Fb(r')),  and each end takes its own partial
//     derivatives.  Writes nb_t (before the fold) and the Poisson adjoint's
//     source from the potential adjoint phib.
//  3. the Poisson adjoint: the fluid-node operator of Eq. 15 is symmetric, so
//     lambda solves L_h lambda = phib with zero wall values, by the same
//     solver as the forward step.
//  4. k_adj_fold: nb_k += -4 pi l_B z_k lambda; sums lambda over time (the
//     electrode potentials enter Poisson linearly, so their gradient is one
//     gather of that sum at the end) and lambda . rho_el for d/dl_B.
#include <math.h>

#include "lbe_device.h"
#include "lbe_internal.h"

namespace lbe {
namespace {

// FP64 values of the stored state: populations and concentrations kept in
// FP64, or as FP32 deviations from w_i rho0 and from the system's n_ref
__device__ __forceinline__ double load_f(const double *f, int i, int idx, int N, double) {
  return f[i * N + idx];
}
__device__ __forceinline__ double load_f(const float *f, int i, int idx, int N, double rho0) {
  return (double)f[i * N + idx] + WQ[i] * rho0;
}
__device__ __forceinline__ double load_n(const double *n, int k, int idx, int N, const double *) {
  return n[k * N + idx];
}
__device__ __forceinline__ double load_n(const float *n, int k, int idx, int N,
                                         const double *ref) {
  return ref[k] + (double)n[k * N + idx];
}

// rho and m = sum_i f_i c_i of the pre-collision populations (the pull of the
// stored array), into rhom[0..3][r]
template <class S>
__global__ __launch_bounds__(BLOCK) void k_adj_moments(Lattice L, Phys P,
                                                       const uint32_t *__restrict__ mask,
                                                       const S *__restrict__ fin,
                                                       double *__restrict__ rhom) {
  const int r = blockIdx.x * BLOCK + threadIdx.x;
  if (r >= L.n) return;
  const uint32_t m = mask[r];
  if (m & SOLID_BIT) return;
  const int N = L.n;
  Offs o;
  site_offsets(L, r, o);
  double f[NQ];
  f[0] = load_f(fin, 0, r, N, P.rho0_d);
#pragma unroll
  for (int i = 1; i < NQ; ++i) {
    const int j = OPP[i];
    // opposite directions share their weight, so either index converts h
    f[i] = solid_link(m, j) ? load_f(fin, j, r, N, P.rho0_d) : load_f(fin, i, nbr(o, r, j), N, P.rho0_d);
  }
  double rho = 0.0, m0 = 0.0, m1 = 0.0, m2 = 0.0;
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    rho += f[i];
    if (CX[i]) m0 += CX[i] * f[i];
    if (CY[i]) m1 += CY[i] * f[i];
    if (CZ[i]) m2 += CZ[i] * f[i];
  }
  rhom[r] = rho;
  rhom[N + r] = m0;
  rhom[2 * N + r] = m1;
  rhom[3 * N + r] = m2;
}

template <int K, class ST>
__global__ __launch_bounds__(BLOCK) void k_adj_fluid(Lattice L, Phys P,
                                                     const uint32_t *__restrict__ mask,
                                                     const double *__restrict__ phi,
                                                     const ST *__restrict__ n,
                                                     const double *__restrict__ rhom,
                                                     const double *__restrict__ abar_in,
                                                     const double *__restrict__ nbar_in,
                                                     double *__restrict__ abar_out,
                                                     double *__restrict__ fbar,
                                                     double *__restrict__ u) {
  const int r = blockIdx.x * BLOCK + threadIdx.x;
  if (r >= L.n) return;
  const uint32_t m = mask[r];
  const int N = L.n;
  // every node stores, a solid one zeros (its slots are never read), so
  // that each store writes whole cache lines
  double ab[NQ], fb0 = 0.0, fb1 = 0.0, fb2 = 0.0, ux = 0.0, uy = 0.0, uz = 0.0;
#pragma unroll
  for (int i = 0; i < NQ; ++i) ab[i] = 0.0;
  if (!(m & SOLID_BIT)) {
    Offs o;
    site_offsets(L, r, o);
    const double ph = phi[r];
    const double *ref = P.nref_d + 4 * system_of(m);
    double nr[K], nbr_r[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      nr[k] = load_n(n, k, r, N, ref);
      nbr_r[k] = nbar_in[k * N + r];
    }
    // force of the link fluxes (as in pass A) and the advective flux's share
    // of the velocity adjoint: sum_i 3 w_i c_i sum_k (nb_k(r') - nb_k(r)) n_k(r);
    // the neighbours' values of nine links at a time loaded before any is used
    double F0 = 0.0, F1 = 0.0, F2 = 0.0, V0 = 0.0, V1 = 0.0, V2 = 0.0;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      double pn[9], nt[9][K], nb[9][K];
#pragma unroll
      for (int j = 0; j < 9; ++j) {
        const int rn = nbr(o, r, 1 + 9 * half + j);
        pn[j] = phi[rn];
#pragma unroll
        for (int k = 0; k < K; ++k) {
          nt[j][k] = load_n(n, k, rn, N, ref);
          nb[j][k] = nbar_in[k * N + rn];
        }
      }
#pragma unroll
      for (int j = 0; j < 9; ++j) {
        const int i = 1 + 9 * half + j;
        if (solid_link(m, i)) continue;
        const double dphi = pn[j] - ph - P.Ec[i];
        double S1, C1;
        sinh_coshm1(dphi, S1, C1);
        double g = 0.0, adv = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          double S, C;
          valence_sc(P.z[k], dphi, S1, C1, S, C);
          g += -((nt[j][k] + nr[k]) * S + (nt[j][k] - nr[k]) * C) * (0.5 / LEN[i]);
          adv += (nb[j][k] - nbr_r[k]) * nr[k];
        }
        const double c = 3.0 * WQ[i] * LEN[i] * g;
        const double a = 3.0 * WQ[i] * adv;
        if (CX[i]) { F0 += CX[i] * c; V0 += CX[i] * a; }
        if (CY[i]) { F1 += CY[i] * c; V1 += CY[i] * a; }
        if (CZ[i]) { F2 += CZ[i] * c; V2 += CZ[i] * a; }
      }
    }
    const double rho = rhom[r], m0 = rhom[N + r], m1 = rhom[2 * N + r], m2 = rhom[3 * N + r];
    const double irho = 1.0 / rho;
    ux = (m0 + 0.5 * F0) * irho;
    uy = (m1 + 0.5 * F1) * irho;
    uz = (m2 + 0.5 * F2) * irho;
    const double uu = ux * ux + uy * uy + uz * uz;
    // adjoint of the collision output: transposed streaming
    double pb[NQ];
    pb[0] = abar_in[r];
#pragma unroll
    for (int i = 1; i < NQ; ++i)
      pb[i] = solid_link(m, i) ? abar_in[OPP[i] * N + r] : abar_in[i * N + nbr(o, r, i)];
    // moments of a_i = pb_i w_i that the collision's derivatives need
    double s0 = 0.0, re = 0.0;
    double s1x = 0.0, s1y = 0.0, s1z = 0.0, sux = 0.0, suy = 0.0, suz = 0.0;
    double sfx = 0.0, sfy = 0.0, sfz = 0.0;
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const double a = pb[i] * WQ[i];
      const double cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
      const double cF = CX[i] * F0 + CY[i] * F1 + CZ[i] * F2;
      s0 += a;
      re += a * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
      if (CX[i]) { s1x += CX[i] * a; sux += CX[i] * a * cu; sfx += CX[i] * a * cF; }
      if (CY[i]) { s1y += CY[i] * a; suy += CY[i] * a * cu; sfy += CY[i] * a * cF; }
      if (CZ[i]) { s1z += CZ[i] * a; suz += CZ[i] * a * cu; sfz += CZ[i] * a * cF; }
    }
    const double beta = 1.0 / P.tau;
    const double gam = 1.0 - 0.5 * beta;
    // d(feq_i)/du and d(source_i)/dF share G = 3 s1 + 9 su - 3 u s0
    const double Gx = 3.0 * s1x + 9.0 * sux - 3.0 * ux * s0;
    const double Gy = 3.0 * s1y + 9.0 * suy - 3.0 * uy * s0;
    const double Gz = 3.0 * s1z + 9.0 * suz - 3.0 * uz * s0;
    const double ubx = beta * rho * Gx + gam * (9.0 * sfx - 3.0 * F0 * s0) + V0;
    const double uby = beta * rho * Gy + gam * (9.0 * sfy - 3.0 * F1 * s0) + V1;
    const double ubz = beta * rho * Gz + gam * (9.0 * sfz - 3.0 * F2 * s0) + V2;
    // u = (m + F/2) / rho
    const double mbx = ubx * irho, mby = uby * irho, mbz = ubz * irho;
    const double rhob = beta * re - (ubx * ux + uby * uy + ubz * uz) * irho;
#pragma unroll
    for (int i = 0; i < NQ; ++i)
      ab[i] = (1.0 - beta) * pb[i] + rhob + (CX[i] * mbx + CY[i] * mby + CZ[i] * mbz);
    fb0 = gam * Gx + 0.5 * mbx;
    fb1 = gam * Gy + 0.5 * mby;
    fb2 = gam * Gz + 0.5 * mbz;
  }
#pragma unroll
  for (int i = 0; i < NQ; ++i) abar_out[i * N + r] = ab[i];
  fbar[r] = fb0;
  fbar[N + r] = fb1;
  fbar[2 * N + r] = fb2;
  u[r] = ux;
  u[N + r] = uy;
  u[2 * N + r] = uz;
}

template <int K, class ST>
__global__ __launch_bounds__(BLOCK) void k_adj_ions(Lattice L, Phys P,
                                                    const uint32_t *__restrict__ mask,
                                                    const double *__restrict__ phi,
                                                    const ST *__restrict__ n,
                                                    const double *__restrict__ u,
                                                    const double *__restrict__ fbar,
                                                    const double *__restrict__ nbar_in,
                                                    double *__restrict__ nbar_out,
                                                    double *__restrict__ src) {
  const int r = blockIdx.x * BLOCK + threadIdx.x;
  if (r >= L.n) return;
  const uint32_t m = mask[r];
  const int N = L.n;
  // every node stores, a solid one zeros (nothing reads them there, and
  // they start at zero), so that each store writes whole cache lines
  double nbo[K], srcv = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) nbo[k] = 0.0;
  if (!(m & SOLID_BIT)) {
    Offs o;
    site_offsets(L, r, o);
    const double ph = phi[r];
    const double ux = u[r], uy = u[N + r], uz = u[2 * N + r];
    const double fx = fbar[r], fy = fbar[N + r], fz = fbar[2 * N + r];
    const double *ref = P.nref_d + 4 * system_of(m);
    double nr[K], nbr_r[K], acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      nr[k] = load_n(n, k, r, N, ref);
      nbr_r[k] = nbar_in[k * N + r];
      acc[k] = 0.0;
    }
    double phib = 0.0;
    // one link's loads at a time: with this kernel's register count,
    // loading nine links ahead (as k_adj_fluid does) halves the occupancy
    // and measured 797 us against 517 us at 192^3
#pragma unroll
    for (int i = 1; i < NQ; ++i) {
      if (solid_link(m, i)) continue;
      const int rn = nbr(o, r, i);
      const double dphi = phi[rn] - ph - P.Ec[i];
      double S1, C1;
      sinh_coshm1(dphi, S1, C1);
      double fs = 0.0, cu = 0.0;
      if (CX[i]) { fs += CX[i] * (fx + fbar[rn]); cu += CX[i] * ux; }
      if (CY[i]) { fs += CY[i] * (fy + fbar[N + rn]); cu += CY[i] * uy; }
      if (CZ[i]) { fs += CZ[i] * (fz + fbar[2 * N + rn]); cu += CZ[i] * uz; }
      const double h = 0.5 / LEN[i];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const double nt = load_n(n, k, rn, N, ref);
        double S, C;
        valence_sc(P.z[k], dphi, S1, C1, S, C);
        const double pbk = nbar_in[k * N + rn] - nbr_r[k];
        const double gb = P.dk[k] * pbk + 3.0 * WQ[i] * LEN[i] * fs;
        // d g / d n(r) = expm1(-delta) / (2 Delta); ideal and advective parts
        acc[k] += gb * (C - S) * h + P.dk[k] * pbk / LEN[i] + pbk * 3.0 * WQ[i] * cu;
        // -z d g / d delta = z [n' e^delta + n e^-delta] / (2 Delta)
        phib += gb * P.z[k] * (nt * (1.0 + C + S) + nr[k] * (1.0 + C - S)) * h;
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) nbo[k] = nbr_r[k] + acc[k];
    // the solver zeroes 6 [sum_i w_i s_i (lambda' - lambda) + src]
    srcv = -phib / 6.0;
  }
#pragma unroll
  for (int k = 0; k < K; ++k) nbar_out[k * N + r] = nbo[k];
  src[r] = srcv;
}

// nb_k += -4 pi l_B z_k lambda; lam_sum += lambda; lam_keep = lambda (warm
// start of the next adjoint solve); block sums of lambda . rho_el
template <int K, class ST>
__global__ __launch_bounds__(BLOCK) void k_adj_fold(Lattice L, Phys P,
                                                    const uint32_t *__restrict__ mask,
                                                    const double *__restrict__ lam,
                                                    const ST *__restrict__ n,
                                                    double *__restrict__ nbar,
                                                    double *__restrict__ lam_sum,
                                                    double *__restrict__ lam_keep,
                                                    double *__restrict__ partial) {
  __shared__ double sm[BLOCK / WAVE];
  const int r = blockIdx.x * BLOCK + threadIdx.x;
  const int N = L.n;
  double v = 0.0;
  const uint32_t m = r < N ? mask[r] : SOLID_BIT;
  if (!(m & SOLID_BIT)) {
    const double l = lam[r];
    const double s = -6.0 * P.src_scale * l;  // -4 pi l_B lambda
    const double *ref = P.nref_d + 4 * system_of(m);
    double q = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      q += P.z[k] * load_n(n, k, r, N, ref);
      nbar[k * N + r] += s * P.z[k];
    }
    lam_sum[r] += l;
    lam_keep[r] = l;
    v = l * q;
  }
  v = block_sum(v, sm);
  if (threadIdx.x == 0) partial[blockIdx.x] = v;
}

// acc[0] += scale * sum of partial[0..nb) (fixed order)
__global__ __launch_bounds__(FINAL) void k_adj_accumulate(const double *__restrict__ partial,
                                                          int nb, double scale,
                                                          double *__restrict__ acc) {
  __shared__ double tree[FINAL];
  const double v = final_sum(partial, nb, tree);
  if (threadIdx.x == 0) acc[0] += scale * v;
}

// Seed of the reverse sweep from the charges, L = sum_e qbar_e Q_e:
//  fluid r:  dL/dphi(r) = q_scale wall sum over links to an electrode node r'
//            of w_i qbar_{e(r')}, added to the adjoint solve's source as -phib/6;
//  solid r:  the explicit derivative -q_scale wall qbar_e sum over links to
//            fluid nodes of w_i (phi_s(r) enters Eq. 16 directly).
__global__ __launch_bounds__(BLOCK) void k_adj_seed(Lattice L, double q_scale,
                                                    const uint32_t *__restrict__ mask,
                                                    const uint8_t *__restrict__ type,
                                                    const double *__restrict__ qbar,
                                                    double *__restrict__ src,
                                                    double *__restrict__ gphis) {
  const int r = blockIdx.x * BLOCK + threadIdx.x;
  if (r >= L.n) return;
  const uint32_t m = mask[r];
  Offs o;
  site_offsets(L, r, o);
  double acc = 0.0;
  if (m & SOLID_BIT) {
    for (int i = 1; i < NQ; ++i)
      if (!solid_link(m, i)) acc += WQ[i];
    gphis[r] = -q_scale * L.wall * qbar[type[r] - 1] * acc;
    return;
  }
  for (int i = 1; i < NQ; ++i)
    if (solid_link(m, i)) acc += WQ[i] * qbar[type[nbr(o, r, i)] - 1];
  gphis[r] = 0.0;
  src[r] += -(q_scale * L.wall * acc) / 6.0;  // after the momentum seed's share
}

// Seed of the momentum term ubar . sum_r (sum_i f_i c_i + F/2) at fluid
// nodes: the population adjoint c_i . ubar and the force adjoint ubar / 2
// (which k_adj_ions then carries to n and phi through the link fluxes).
__global__ __launch_bounds__(BLOCK) void k_adj_seed_momentum(Lattice L,
                                                             const uint32_t *__restrict__ mask,
                                                             double ux, double uy, double uz,
                                                             double *__restrict__ abar,
                                                             double *__restrict__ fbar) {
  const int r = blockIdx.x * BLOCK + threadIdx.x;
  if (r >= L.n || (mask[r] & SOLID_BIT)) return;
  const int N = L.n;
#pragma unroll
  for (int i = 0; i < NQ; ++i) abar[i * N + r] = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
  fbar[r] = 0.5 * ux;
  fbar[N + r] = 0.5 * uy;
  fbar[2 * N + r] = 0.5 * uz;
}

// gphis(r) += -6 wall sum over links to fluid nodes r' of w_i lam_sum(r'):
// the transpose of the wall term that phi_s contributes to Eq. 15
__global__ __launch_bounds__(BLOCK) void k_adj_phis(Lattice L, const uint32_t *__restrict__ mask,
                                                    const double *__restrict__ lam_sum,
                                                    double *__restrict__ gphis) {
  const int r = blockIdx.x * BLOCK + threadIdx.x;
  if (r >= L.n) return;
  const uint32_t m = mask[r];
  if (!(m & SOLID_BIT)) return;
  Offs o;
  site_offsets(L, r, o);
  double acc = 0.0;
  for (int i = 1; i < NQ; ++i)
    if (!solid_link(m, i)) acc += WQ[i] * lam_sum[nbr(o, r, i)];
  gphis[r] += -6.0 * L.wall * acc;
}

}  // namespace

#define LBE_DISPATCH_K(K, CALL) \
  switch (K) {                  \
    case 1: CALL(1); break;     \
    case 2: CALL(2); break;     \
    case 3: CALL(3); break;     \
    default: CALL(4); break;    \
  }

template <class S>
hipError_t launch_adj_moments(hipStream_t s, const Lattice &L, const Phys &P,
                              const uint32_t *mask, const S *fin, double *rhom) {
  hipLaunchKernelGGL(k_adj_moments<S>, dim3(blocks_for(L.n)), dim3(BLOCK), 0, s, L, P, mask, fin,
                     rhom);
  return hipGetLastError();
}

template <class S>
hipError_t launch_adj_fluid(hipStream_t s, const Lattice &L, const Phys &P, const uint32_t *mask,
                            const double *phi, const S *n, const double *rhom,
                            const double *abar_in, const double *nbar_in, double *abar_out,
                            double *fbar, double *u) {
#define CALL(KK)                                                                     \
  hipLaunchKernelGGL((k_adj_fluid<KK, S>), dim3(blocks_for(L.n)), dim3(BLOCK), 0, s, L, P, \
                     mask, phi, n, rhom, abar_in, nbar_in, abar_out, fbar, u)
  LBE_DISPATCH_K(P.K, CALL)
#undef CALL
  return hipGetLastError();
}

template <class S>
hipError_t launch_adj_ions(hipStream_t s, const Lattice &L, const Phys &P, const uint32_t *mask,
                           const double *phi, const S *n, const double *u, const double *fbar,
                           const double *nbar_in, double *nbar_out, double *src) {
#define CALL(KK)                                                                    \
  hipLaunchKernelGGL((k_adj_ions<KK, S>), dim3(blocks_for(L.n)), dim3(BLOCK), 0, s, L, P, \
                     mask, phi, n, u, fbar, nbar_in, nbar_out, src)
  LBE_DISPATCH_K(P.K, CALL)
#undef CALL
  return hipGetLastError();
}

template <class S>
hipError_t launch_adj_fold(hipStream_t s, const Lattice &L, const Phys &P, const uint32_t *mask,
                           const double *lam, const S *n, double *nbar, double *lam_sum,
                           double *lam_keep, double *partial, double *lb_acc) {
  const int nb = (int)blocks_for(L.n);
#define CALL(KK)                                                                             \
  hipLaunchKernelGGL((k_adj_fold<KK, S>), dim3(nb), dim3(BLOCK), 0, s, L, P, mask, lam, n, nbar, \
                     lam_sum, lam_keep, partial)
  LBE_DISPATCH_K(P.K, CALL)
#undef CALL
  // dL/dl_B gathers -4 pi lambda . rho_el from every reverse step
  hipLaunchKernelGGL(k_adj_accumulate, dim3(1), dim3(FINAL), 0, s, partial, nb, -4.0 * M_PI,
                     lb_acc);
  return hipGetLastError();
}

#define LBE_ADJ_INSTANTIATE(S)                                                                   \
  template hipError_t launch_adj_moments<S>(hipStream_t, const Lattice &, const Phys &,         \
                                            const uint32_t *, const S *, double *);             \
  template hipError_t launch_adj_fluid<S>(hipStream_t, const Lattice &, const Phys &,           \
                                          const uint32_t *, const double *, const S *,          \
                                          const double *, const double *, const double *,       \
                                          double *, double *, double *);                        \
  template hipError_t launch_adj_ions<S>(hipStream_t, const Lattice &, const Phys &,            \
                                         const uint32_t *, const double *, const S *,           \
                                         const double *, const double *, const double *,        \
                                         double *, double *);                                   \
  template hipError_t launch_adj_fold<S>(hipStream_t, const Lattice &, const Phys &,            \
                                         const uint32_t *, const double *, const S *, double *, \
                                         double *, double *, double *, double *);
LBE_ADJ_INSTANTIATE(double)
LBE_ADJ_INSTANTIATE(float)
#undef LBE_ADJ_INSTANTIATE

hipError_t launch_adj_seed(hipStream_t s, const Lattice &L, double q_scale, const uint32_t *mask,
                           const uint8_t *type, const double *qbar, double *src, double *gphis) {
  hipLaunchKernelGGL(k_adj_seed, dim3(blocks_for(L.n)), dim3(BLOCK), 0, s, L, q_scale, mask, type,
                     qbar, src, gphis);
  return hipGetLastError();
}

hipError_t launch_adj_seed_momentum(hipStream_t s, const Lattice &L, const uint32_t *mask,
                                    const double *ubar, double *abar, double *fbar) {
  hipLaunchKernelGGL(k_adj_seed_momentum, dim3(blocks_for(L.n)), dim3(BLOCK), 0, s, L, mask,
                     ubar[0], ubar[1], ubar[2], abar, fbar);
  return hipGetLastError();
}

hipError_t launch_adj_phis(hipStream_t s, const Lattice &L, const uint32_t *mask,
                           const double *lam_sum, double *gphis) {
  hipLaunchKernelGGL(k_adj_phis, dim3(blocks_for(L.n)), dim3(BLOCK), 0, s, L, mask, lam_sum,
                     gphis);
  return hipGetLastError();
}

}  // namespace lbe
