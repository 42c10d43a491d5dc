// lbe_internal.h -- declarations shared by the host driver and the HIP
// kernels of the LBE library (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbe {

// D3Q19 (Sec. II B of arXiv:1907.04732) in the order documented in lbe.h.
constexpr int NQ = 19;
constexpr int CX[NQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[NQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[NQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
// opposite direction: pairs (1,2), (3,4), ... (17,18)
constexpr int OPP[NQ] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
constexpr double W0 = 1.0 / 3.0, W1 = 1.0 / 18.0, W2 = 1.0 / 36.0;
constexpr double WQ[NQ] = {W0, W1, W1, W1, W1, W1, W1, W2, W2, W2, W2,
                           W2, W2, W2, W2, W2, W2, W2, W2};
constexpr double SQRT2 = 1.4142135623730951;
// link length |c_i| (Delta_i of Eq. 10)
constexpr double LEN[NQ] = {0.0, 1, 1, 1, 1, 1, 1, SQRT2, SQRT2, SQRT2, SQRT2,
                            SQRT2, SQRT2, SQRT2, SQRT2, SQRT2, SQRT2, SQRT2, SQRT2};
// lattice factor A0 = 1 + 2 sqrt(2) of Eq. 9 (D3Q19)
constexpr double A0 = 1.0 + 2.0 * SQRT2;

// Per-node flag word: bit (i-1), i = 1..18, set when the neighbour r + c_i
// is solid; bit 31 set when the node itself is solid.
constexpr uint32_t SOLID_BIT = 1u << 31;
// Bits 18..30 of a fluid node's flag word: the index of the independent
// system it belongs to (batched runs; 0 otherwise).
constexpr int SYS_SHIFT = 18;
constexpr uint32_t SYS_MASK = 0x1fffu;
constexpr int MAX_SYSTEMS = 8192;
__host__ __device__ inline int system_of(uint32_t m) { return (int)((m >> SYS_SHIFT) & SYS_MASK); }

// Accelerator complex dies (XCDs) of the part, each with its own L2; the
// hardware hands out the blocks of a launch round-robin over them.
constexpr int NXCD = 8;

struct Lattice {
  int nx, ny, nz;
  int nxy;
  int n;            // sites
  uint32_t selfm;   // bit (i-1) set when link i maps a node onto itself
  double wall;      // factor on a solid-fluid link: 2 (Eq. 15) or 1 (first-order scheme)
  int xcd;          // 1: stencil kernels give each XCD a contiguous run of blocks
  double rnx, rnxy; // 1 / nx and 1 / nxy: site coordinates by multiplication
};

// Every field of a lattice, the reciprocals included (the kernels take a
// site's coordinates from them).
inline Lattice make_lattice(int nx, int ny, int nz, uint32_t selfm, double wall, int xcd) {
  Lattice L{};
  L.nx = nx;
  L.ny = ny;
  L.nz = nz;
  L.nxy = nx * ny;
  L.n = nx * ny * nz;
  L.selfm = selfm;
  L.wall = wall;
  L.xcd = xcd;
  L.rnx = 1.0 / nx;
  L.rnxy = 1.0 / ((double)nx * ny);
  return L;
}

// Step passes on LDS-staged tiles, selected by TB_TILED as a pass's launch
// shape (the context's timing picks it where the tiles fit the lattice):
// pass B on blocks of TILE_X x TILE_Y nodes marching through TILE_Z planes
// along z (tiles_fit), pass A on the plane rings below (rings_fit).  On the
// 192^3 porous electrode pass B took 191 us on 64 x 4 x 16 tiles, 187 us
// with the tiles of a run of planes given to one die in consecutive chunks,
// and 185 us on 32 x 8 x 8 tiles in that order (199 us without it).
constexpr int TILE_X = 32, TILE_Y = 8, TILE_Z = 8;  // the plane rings' tiles (below)
constexpr int TB_TILED = 1;
inline bool tiles_fit(const Lattice &L) { return L.nx % TILE_X == 0 && L.ny % TILE_Y == 0; }

// Physical constants of one context, passed by value to the kernels.
struct Phys {
  int K;                 // species
  int z[4];
  double dk[4];          // D_k / A0
  double Ec[NQ];         // E_app . c_i
  double tau;
  double src_scale;      // 4 pi l_B / 6
  double omega;
  // mixed form: references of the deviation storage, per system s
  double rho0_d;         // rest density rho0
  const double *nref_d;  // n_ref,k of system s at [4 s + k] (device)
  const float *nref_f;   // the same in FP32 (device)
  const double *qref;    // sum_k z_k n_ref,k of system s at [s] (device)
  float rho0_f, itau_f;
  float dk_f[4];
  int unit_z;            // every species has |z| = 1 (the mixed form's fast link loop)
};

// One multigrid level (cell-centred; spacing h = 2^level in fine units).
struct MgLevel {
  int nx, ny, nz, nxy, n;
  uint32_t selfm;
  double h2, inv_h2;
  double wall;      // as Lattice::wall
  double rnx, rnxy; // 1 / nx and 1 / nxy: cell coordinates by multiplication
  int xcd;          // as Lattice::xcd
};

inline MgLevel make_level(int nx, int ny, int nz, uint32_t selfm, double h2, double wall,
                          int xcd) {
  return MgLevel{nx, ny, nz, nx * ny, nx * ny * nz, selfm, h2, 1.0 / h2, wall,
                 1.0 / nx, 1.0 / ((double)nx * ny), xcd};
}

// The multigrid stencil kernels' plane-ring form: LDS-staged tiles of
// RING_TX x RING_TY cells (a wavefront holds two rows), each block marching
// along z through a run of zrun planes, on a level whose nx and ny are
// multiples of the tile's.  A run takes RING_ZRUN planes, or fewer so that
// the launch keeps RING_MIN_BLOCKS blocks, but not fewer than RING_MIN_ZRUN
// (each run reloads two planes around it); below that the level is too small
// for the form and ring_zrun returns 0.  (On the 192^3 lattice runs of 16,
// 8, 4 and 2 planes gave the finest-level kernels 1728, 3456, 6912 and
// 13824 blocks; 8 was the fastest.  On the 160 x 160 x 64 cell runs of 8
// planes, 800 blocks, were slower than runs of 4, and the 96^3 level gained
// nothing from runs of 4 in 864 blocks.)  A launcher's `ring` is RING_OFF,
// RING_AUTO (that rule) or a run length forced (> 0, on levels that fit).
constexpr int RING_TX = 32, RING_TY = 8;
static_assert(TILE_X == RING_TX && TILE_Y == RING_TY, "pass B's tiles are the plane rings' tiles");
constexpr int RING_ZRUN = 8, RING_MIN_BLOCKS = 1024, RING_MIN_ZRUN = 4;
constexpr int RING_OFF = -1, RING_AUTO = 0;
inline int ring_zrun(const MgLevel &lv, int ring) {  // 0: the gathering kernels
  if (ring == RING_OFF || lv.nx % RING_TX || lv.ny % RING_TY) return 0;
  if (ring > 0) return ring;
  const long tiles = (long)(lv.nx / RING_TX) * (lv.ny / RING_TY);
  for (int zr = RING_ZRUN; zr >= RING_MIN_ZRUN; zr /= 2)
    if (tiles * ((lv.nz + zr - 1) / zr) >= RING_MIN_BLOCKS) return zr;
  return 0;
}
inline bool rings_fit(const Lattice &L) { return L.nx % RING_TX == 0 && L.ny % RING_TY == 0; }
inline int ring_blocks(const MgLevel &lv, int zrun) {
  return (lv.nx / RING_TX) * (lv.ny / RING_TY) * ((lv.nz + zrun - 1) / zrun);
}
// The restriction from a fine level in that form: each coarse cell's
// children are pairs of neighbours along x, y (within a wavefront) and z
// (consecutive planes of a run), so the fine level needs even sizes and
// the run an even length.
inline int ring_zrun_restrict(const MgLevel &f, int ring) {
  if (f.nz % 2) return 0;
  const int zr = ring_zrun(f, ring);
  return zr + (zr & 1);
}

// Fine level f -> coarse level c: coarse cell (X, Y, Z) holds the fine cells
// whose shifted indices ((x - ox) mod nx, ...) are (2X or 2X+1, ...).
struct MgTransfer {
  MgLevel f, c;
  int ox, oy, oz;
};

// Device-side control of one Poisson solve.  The residual check sets `done`
// once ||R||_inf <= tol (or the residual is not finite); every kernel of the
// solve returns at once when `done` is set, so the host can queue a predicted
// number of sweeps or cycles and wait once.  Every check also publishes the
// block to `mirror`, a host-mapped copy the host polls instead of copying the
// block back and synchronising the stream.
struct SolveCtl {
  double resid;   // last residual inf-norm
  double tol;     // <= 0: never done (fixed iteration count)
  int done;
  int iters;      // sweeps or cycles completed when done was set
  int checks;     // residual evaluations so far
  int nonfinite;  // the residual was NaN or Inf
  int count;      // sweeps or cycles completed so far (each check adds its unit)
  int seq;        // which solve of the context this is (set by the host)
  // published to the mirror in one 8-byte store after the values above:
  // seq << 32 | done << 31 | checks, so the host never pairs a stop flag or
  // check count of one solve (or check) with another
  unsigned long long stamp;
  SolveCtl *mirror;  // host-mapped copy (device address), or null
};

// Outcome of a run of graph-replayed time steps (lbe_step_chunk), folded by
// every step after its solve; zeroed by the host before the run.
struct ChunkStatus {
  double resid_max;  // largest final residual of the steps' solves
  long long iters;   // sweeps or cycles summed over the steps
  int unconverged;   // steps whose solve ended above the tolerance
  int nonfinite;     // steps whose residual was NaN or Inf
};

// Flexible conjugate gradients preconditioned by one V-cycle (device state).
struct KrylovCtl {
  double alpha, beta;
  double pq_prev;  // (p, A p) of the previous direction
  int first;       // 1 until the first direction of a solve is formed
  int pad;
};

// The coarse end of the hierarchy handled by one work-group in LDS.
constexpr int MG_MAX_SMALL = 8;
constexpr int MG_MAX_DENSE = 512;         // largest coarsest level solved with a dense inverse
constexpr int MG_GROUP_SCAN = 1 << 16;    // levels up to this size keep host copies of their cells
struct MgSmall {
  int nlev;                               // levels in the set; the last is the coarsest
  MgLevel lv[MG_MAX_SMALL];
  MgTransfer tr[MG_MAX_SMALL];            // tr[k]: level k-1 -> k, k >= 1
  const uint32_t *mask[MG_MAX_SMALL];
  int off_e[MG_MAX_SMALL], off_r[MG_MAX_SMALL], off_m[MG_MAX_SMALL];  // LDS offsets (elements)
  int off_e2[MG_MAX_SMALL];               // second Jacobi buffer per level
  int off_x;                              // compact right-hand side of the exact solve (T)
  int nu1, nu2;
  int nf;                                 // coarsest exact solve: fluid cells,
  const void *ainv;                       // inverse (column-major), cell of each row
  const int *fcell;
  int coarse_sweeps;
  double omega;
  double jacobi;                          // > 0: Jacobi smoothing with this weight, else GS
  // independent groups, one work-group each (batched systems):
  // groups[2 (k G + g)] and groups[2 (k G + g) + 1] are the first cell and the
  // length of group g's cyclic range on level k; row k = nlev holds the first
  // fluid row and the row count of the group in the exact solve; null: one
  // group, whole levels
  int ngroups;
  const int *groups;
};

enum KernelKind {
  KK_FLUID = 0,   // link fluxes, force, LB collide/stream (pull); writes u, n*
  KK_IONS,        // advective ion fluxes, n(t+1), Poisson source (and the warm start)
  KK_SOR,         // one colour of the FP64 SOR sweep
  KK_RESID,       // FP64 residual inf-norm
  KK_CHARGE,      // electrode charges
  KK_TOTALS,      // conserved totals
  KK_OBSERVE,     // pre-collision populations and velocity
  KK_SOR32,       // one colour of the FP32 correction sweep
  KK_CORRECT,     // phi += e
  KK_MG_RESID,    // outer FP64 residual feeding the multigrid correction
  KK_MG_SMOOTH,   // one colour of the smoother on a coarse level
  KK_MG_SMOOTH0,  // one colour of the smoother on the finest level
  KK_MG_RESTRICT, // residual + restriction to the next level
  KK_MG_PROLONG,  // trilinear prolongation + correction
  KK_MG_COARSE,   // coarsest-level solve in one work-group
  KK_MG_SMALL,    // the coarse levels of a V-cycle in one work-group
  KK_FCG_APPLY,   // Krylov: A z and the sums that give beta and alpha
  KK_FCG_UPDATE,  // Krylov: p, q = A p, phi += alpha p, r -= alpha q, stop check
  KK_ADJ_FLUID,   // reverse step: streaming, collision and velocity adjoints
  KK_ADJ_IONS,    // reverse step: link-flux and force adjoints, Poisson-adjoint source
  KK_ADJ_FOLD,    // reverse step: fold the Poisson adjoint into the ion adjoint
  KK_ADJ_SEED,    // reverse sweep: seed from the charge weights; phi_s gradient
  KK_ADJ_MOMENTS, // reverse sweep: rho and m of a recomputed state
  KK_REWIND,      // back to the start of a step whose solve failed
  KK_EXPAND_N,    // mixed form: FP64 concentrations into a caller's device buffer
  KK_MG_SMOOTH0_PHI,  // the finest level's last Jacobi sweep of a cycle, with phi += e
  KK_MOMENTUM,    // total fluid momentum
  KK_COUNT
};

extern const char *const kKernelNames[KK_COUNT];

// ---- launchers (lbe_kernels.hip) -----------------------------------------
// All take the stream; they return hipSuccess or the launch error.
// Step pass A: link fluxes, force, collide-stream; writes f', u and
// n* = n - (diffusion-migration outflow) into nstar.
hipError_t launch_fluid_f64(hipStream_t s, const Lattice &L, const Phys &P, const uint32_t *mask,
                            const double *phi, const double *n, const double *fin, double *fout,
                            double *u, double *nstar, int tb, bool nt);
// tb: block size of the step passes (128, 256 or 512); nt: non-temporal streams.
// Step pass B: advective outflow with u; nio holds n* on entry, n(t+1) on exit.
// With prev = [phi(t-1) | phi(t-2)] (2 N; NULL: none) it also moves phi to
// its extrapolation in time of the given order (0 constant, 1 linear, 2
// quadratic) as the next solve's start, and shifts the history; order -1
// (prev: N) only copies phi(t) into prev.
hipError_t launch_ions_f64(hipStream_t s, const Lattice &L, const Phys &P, const uint32_t *mask,
                           const double *u, const double *n, double *nio, double *src, int order,
                           double *phi, double *prev, int tb, bool nt);
// A step's solve failed: phi = prev[0..N) (phi(t), kept by pass B), the
// source recomputed from n(t), and with shift prev[0..N) = prev[N..2N)
// (the extrapolation history back by one step).  Fluid nodes only.
hipError_t launch_rewind_f64(hipStream_t s, const Lattice &L, const Phys &P, const uint32_t *mask,
                             const double *n, double *src, double *phi, double *prev, int shift);
// dst[idx[t]] = val[t] for t < count (new solid-node potentials)
hipError_t launch_scatter(hipStream_t s, int count, const int *idx, const double *val,
                          double *dst);
hipError_t launch_sor_f64(hipStream_t s, const Lattice &L, const Phys &P, int colour,
                          const uint32_t *mask, const double *src, double *phi,
                          const SolveCtl *ctl);
// residual inf-norm over fluid nodes into *out (device); partial is scratch
// of size >= residual_blocks(L)
int residual_blocks(const Lattice &L);
// residual check after `add` more iterations: ||R||_inf into ctl->resid;
// sets ctl->done (with iters = the iterations counted so far)
hipError_t launch_resid_f64(hipStream_t s, const Lattice &L, const uint32_t *mask,
                            const double *src, const double *phi, double *partial, SolveCtl *ctl,
                            int add);
// Start of a solve queued without the host: the control block cleared on
// the device (tolerance tol, no host-mapped copy), one thread.
hipError_t launch_ctl_reset(hipStream_t s, SolveCtl *ctl, double tol);
// Fold the finished solve in ctl into st (one thread).
hipError_t launch_chunk_status(hipStream_t s, const SolveCtl *ctl, ChunkStatus *st);
// gate (may be NULL): both kernels return at once unless gate->done is set
hipError_t launch_charge(hipStream_t s, const Lattice &L, double q_scale, const uint32_t *mask,
                         const double *phi, const int *iface_site, const int *blk_elec,
                         const int *blk_begin, const int *blk_end, int nblocks, int ne,
                         double *partial, double *out, const SolveCtl *gate);
hipError_t launch_totals_f64(hipStream_t s, const Lattice &L, int K, const int *z,
                             const uint32_t *mask, const double *fin, const double *n,
                             double *partial, double *out /*2+K*/);
// Records msg for lbe_last_error(NULL) and returns code (calls without a
// context).
int report_init_error(int code, const char *msg);

hipError_t launch_momentum(hipStream_t s, const Lattice &L, const uint32_t *mask,
                           const double *fpre, const double *u, double *partial, double *out);
hipError_t launch_observe_f64(hipStream_t s, const Lattice &L, const Phys &P,
                              const uint32_t *mask, const double *phi, const double *n,
                              const double *fin, double *fpre, double *u);
int totals_blocks(const Lattice &L);

// mixed form (lbe_kernels_f32.hip): h = f - w rho0 in FP32, nu = n - n_ref as
// the FP32 pair nu + lo.  Pass A writes its increment into dnu; pass B adds
// it and its own to (nu, lo_in), writing the new pair to (nuio, lo_out).
hipError_t launch_fluid_f32(hipStream_t s, const Lattice &L, const Phys &P, const uint32_t *mask,
                            const double *phi, const float *nu, const float *hin, float *hout,
                            float *u, float *dnu, int tb, bool nt);
hipError_t launch_ions_f32(hipStream_t s, const Lattice &L, const Phys &P, const uint32_t *mask,
                           const float *u, const float *nu, const float *lo_in, float *nuio,
                           float *lo_out, double *src, int order, double *phi, double *prev,
                           int tb, bool nt);
hipError_t launch_observe_f32(hipStream_t s, const Lattice &L, const Phys &P,
                              const uint32_t *mask, const double *phi, const float *nu,
                              const float *hin, double *fpre, double *u);
hipError_t launch_rewind_f32(hipStream_t s, const Lattice &L, const Phys &P, const uint32_t *mask,
                             const float *nu, const float *lo, double *src, double *phi,
                             double *prev, int shift);
// n = n_ref + (nu + lo) (K N doubles, species-major; 0 on solid nodes)
hipError_t launch_expand_n_f32(hipStream_t s, const Lattice &L, const Phys &P,
                               const uint32_t *mask, const float *nu, const float *lo, double *n);
hipError_t launch_totals_f32(hipStream_t s, const Lattice &L, const Phys &P, const uint32_t *mask,
                             const float *hin, const float *nu, const float *lo, double *partial,
                             double *out);

// reverse mode (lbe_adjoint.hip).  S: storage of the recomputed state,
// double (FP64 form) or float (mixed form: h = f - w rho0, nu = n - n_ref).
// rho and momentum of the pulled populations into rhom (4 N)
template <class S>
hipError_t launch_adj_moments(hipStream_t s, const Lattice &L, const Phys &P,
                              const uint32_t *mask, const S *fin, double *rhom);
// abar_in/nbar_in: adjoints at t+1; writes abar_out, the force adjoint and u
template <class S>
hipError_t launch_adj_fluid(hipStream_t s, const Lattice &L, const Phys &P, const uint32_t *mask,
                            const double *phi, const S *n, const double *rhom,
                            const double *abar_in, const double *nbar_in, double *abar_out,
                            double *fbar, double *u);
// writes nbar_out (before the Poisson fold) and src = -phib/6
template <class S>
hipError_t launch_adj_ions(hipStream_t s, const Lattice &L, const Phys &P, const uint32_t *mask,
                           const double *phi, const S *n, const double *u, const double *fbar,
                           const double *nbar_in, double *nbar_out, double *src);
// with lam the Poisson adjoint: nbar += -4 pi l_B z lam, lam_sum += lam,
// lam_keep = lam, *lb_acc += -4 pi sum lam rho_el (partial: residual_blocks(L))
template <class S>
hipError_t launch_adj_fold(hipStream_t s, const Lattice &L, const Phys &P, const uint32_t *mask,
                           const double *lam, const S *n, double *nbar, double *lam_sum,
                           double *lam_keep, double *partial, double *lb_acc);
// charge seed: adds its share of the adjoint source to src (solid entries
// untouched), writes the explicit phi_s gradient
hipError_t launch_adj_seed(hipStream_t s, const Lattice &L, double q_scale, const uint32_t *mask,
                           const uint8_t *type, const double *qbar, double *src, double *gphis);
// momentum seed (ubar: 3 host values): abar = c_i . ubar, fbar = ubar / 2 on fluid nodes
hipError_t launch_adj_seed_momentum(hipStream_t s, const Lattice &L, const uint32_t *mask,
                                    const double *ubar, double *abar, double *fbar);
hipError_t launch_adj_phis(hipStream_t s, const Lattice &L, const uint32_t *mask,
                           const double *lam_sum, double *gphis);

// multigrid (lbe_mg.hip); T = double (FP64 form) or float (mixed form).
// `ring` selects the plane-ring form of a stencil kernel (ring_zrun): the
// same values per cell, and in launch_fcg_apply the Krylov sums in another
// (fixed) order.
// FP64 residual check; writes the correction's right-hand side r0 and its
// start e0: 0, or with jacobi > 0 the result of one Jacobi sweep of that
// weight from 0 (pointwise), so a V-cycle can skip its first sweep
template <class T>
hipError_t launch_mg_outer_resid(hipStream_t s, const MgLevel &lv, const uint32_t *mask,
                                 const double *src, const double *phi, T *r0, T *e0,
                                 double *partial, SolveCtl *ctl, int add, double *r64,
                                 KrylovCtl *kc, double jacobi, int ring);
// Flexible CG on A e = R (A = -L_h, level 0), preconditioner z = V-cycle(r):
//   beta = -(z, q_prev) / (p_prev, q_prev) (0 for the first direction),
//   p = z + beta p,  q = A p,  alpha = (r, p) / (p, q),
//   phi += alpha p,  r -= alpha q  (r also copied to r0 in T, e0 zeroed),
// then the stop check on ||r||_inf.  The directions p, q are held in T (the
// correction's precision; phi and r stay FP64 and move along the stored
// vectors).  Two passes: launch_fcg_apply forms A z
// (into az) and the sums from which beta, (p, q) = (z, A z) + 2 beta (z, q') +
// beta^2 (p', q') and (r, p) = (r, z) + beta (r, p') follow; launch_fcg_update
// writes p = z + beta p', q = A z + beta q', updates phi and r and checks.
template <class T>
hipError_t launch_fcg_apply(hipStream_t s, const MgLevel &lv, const uint32_t *mask, const T *z,
                            const T *q_prev, const T *p_prev, const double *r,
                            double *az, double *partial, KrylovCtl *kc, const SolveCtl *ctl,
                            int ring);
template <class T>
hipError_t launch_fcg_update(hipStream_t s, int n, const uint32_t *mask, const T *z,
                             const double *az, T *p, T *q, double *phi, double *r,
                             T *r0, T *e0, double *partial, const KrylovCtl *kc, SolveCtl *ctl,
                             int add, const MgLevel &lv,
                             double jac);  // jac > 0: e0 gets lv's first Jacobi sweep
template <class T>
hipError_t launch_mg_smooth(hipStream_t s, const MgLevel &lv, double omega, int colour,
                            const uint32_t *mask, const T *rhs, T *e, const SolveCtl *ctl);
// damped Jacobi sweep x_in -> x_out (different arrays):
// x <- x + omega ([sum w s x' + hs rhs] / sum w s - x); with phi_add the
// result is also added to phi on fluid cells, as launch_mg_correct does
template <class T>
hipError_t launch_jacobi(hipStream_t s, const MgLevel &lv, double omega, double hs,
                         const uint32_t *mask, const T *rhs, const T *x_in, T *x_out,
                         const SolveCtl *ctl, double *phi_add, int ring);
template <class T>
hipError_t launch_mg_restrict(hipStream_t s, const MgTransfer &tr, const uint32_t *mf,
                              const uint32_t *mc, const T *rf, const T *ef, T *rc, T *ec,
                              const SolveCtl *ctl, bool tiled, double jac = 0.0, double hs = 0.0,
                              int ring = RING_OFF);
// tiled: k_restrict_tiled where it applies; jac > 0: ec receives the coarse
// level's first damped Jacobi sweep (relaxation jac, hs = h^2/6) from zero
// instead of zero
template <class T>
hipError_t launch_mg_prolong(hipStream_t s, const MgTransfer &tr, const uint32_t *mf,
                             const uint32_t *mc, const T *ec, T *ef, const SolveCtl *ctl,
                             int ring = RING_OFF);
template <class T>
hipError_t launch_mg_coarse(hipStream_t s, const MgLevel &lv, double omega, double jacobi,
                            int sweeps, const uint32_t *mask, const T *rhs, T *e, T *e2,
                            const SolveCtl *ctl);
template <class T>
hipError_t launch_mg_correct(hipStream_t s, int n, const uint32_t *mask, const T *e, double *phi,
                             const SolveCtl *ctl);
// coarse end of a V-cycle in one work-group; r_in/e_out on the set's finest level
template <class T>
hipError_t launch_mg_small(hipStream_t s, const MgSmall &S, size_t lds_bytes, const T *r_in,
                           T *e_out, const SolveCtl *ctl);
template <class T>
hipError_t prepare_mg_small(size_t lds_bytes);
// coarsest level by a dense precomputed inverse over its nf fluid cells
template <class T>
hipError_t launch_mg_coarse_dense(hipStream_t s, int nf, const T *ainv, const int *fcell,
                                  const T *rhs, T *e, const SolveCtl *ctl);

}  // namespace lbe
