// lbe_capi.cpp -- the C ABI of include/lbe.h: parameter and geometry
// checks, device state, and the per-step driver that sequences the kernels of
// lbe_kernels.hip on one HIP stream.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <string>
#include <vector>

#include "../../include/lbe.h"
#include "lbe_internal.h"

using namespace lbe;

// Whole time steps captured in one graph by lbe_step_chunk (even, so that a
// replay ends on the buffer parity it started from).
constexpr int CHUNK_STEPS = 16;

struct lbe_ctx {
  lbe_params p{};
  Lattice L{};
  Phys P{};
  int K = 0, ne = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;

  // device state (FP64 form)
  uint32_t *mask = nullptr;
  double *phi = nullptr, *src = nullptr, *u = nullptr;
  double *phi_prev = nullptr;  // converged phi(t-1), phi(t-2) (LBE_EXTRAPOLATE, 2 N)
  int extrap_hist = 0;         // how many of the two are valid
  double *phi_keep = nullptr;  // phi(t) as the step started (N; without LBE_EXTRAPOLATE)
  double *n[2] = {nullptr, nullptr};
  double *f[2] = {nullptr, nullptr};
  // mixed form: FP32 deviations h = f - w rho0, nu = n - n_ref held as the
  // pair nu32 + lo32 (lo32 only read and written by a node's own update),
  // FP32 velocity
  float *h32[2] = {nullptr, nullptr};
  float *nu32[2] = {nullptr, nullptr};
  float *lo32[2] = {nullptr, nullptr};
  float *u32 = nullptr;
  double *obs = nullptr;  // FP64 scratch for observables of the mixed form (22 N)
  bool mixed = false;
  std::vector<uint8_t> type_h;  // node types (host copy)
  int cur = 0;

  // reductions
  double *partial = nullptr;
  double *dout = nullptr;  // small device results (totals)
  double *hpin = nullptr;  // pinned host mirror of dout
  SolveCtl *ctl = nullptr;    // device control block of the running Poisson solve
  SolveCtl *ctl_h = nullptr;  // pinned host copy of it (what the driver reads)
  SolveCtl *ctl_pub = nullptr;  // host-mapped copy the checks publish to (coherent)
  SolveCtl *ctl_pub_d = nullptr;  // its device address
  int checks_queued = 0;        // residual checks queued in the running solve
  int seq = 0;                  // solves started (the running one's stamp)
  int pred_iters = 0;         // iterations the last time-step solve needed
  bool use_graphs = true;     // replay one solver unit as a captured HIP graph
  bool tiles = true;          // the row-order (LDS-combined) restriction where it applies
  int rings = RING_AUTO;      // plane-ring stencil kernels (RING_OFF, RING_AUTO, a run length)
  bool coarse_start = true;   // restriction writes the coarse level's first Jacobi sweep
  int tb_a = 256, tb_b = 256;  // block sizes of the step passes A and B (tuned at init)
  bool nt_a = false, nt_b = false;  // non-temporal streams in passes A and B (set at init)
  // a time step's charge row: queued by the solve right after its predicted
  // units, gated on convergence, so it runs while the host waits
  double *charge_dst = nullptr;
  bool charge_queued = false;
  hipGraphExec_t unit_exec = nullptr;
  // graph-replayed steps (lbe_step_chunk): CHUNK_STEPS whole steps captured
  // for one unit count, buffer parity and tolerance; each step's charges
  // staged in chunk_q and its outcome folded into chunk_st
  hipGraphExec_t chunk_exec = nullptr;
  int chunk_units = 0, chunk_cur = -1;
  double chunk_tol = 0.0;
  int queue_units = 0;  // > 0 while a chunk is captured: fixed units, no host reads
  double *chunk_q = nullptr;
  ChunkStatus *chunk_st = nullptr;

  // electrode charge tables
  int *iface = nullptr, *blk_elec = nullptr, *blk_begin = nullptr, *blk_end = nullptr;
  // flexible-CG state (LBE_KRYLOV): residual (FP64), direction and its image
  // (in the correction's precision: FP32 in the mixed form, in buffers sized
  // for FP64)
  double *kr = nullptr, *kp = nullptr, *kq = nullptr;
  double *kaz = nullptr;  // A z of the current iteration
  KrylovCtl *kc = nullptr;
  // per-system references of the mixed form (device tables) and each node's system
  std::vector<uint16_t> sys_h;
  double *nref_d_tab = nullptr, *qref_tab = nullptr;
  float *nref_f_tab = nullptr;
  std::vector<double> nref_h;  // host copy, [4 s + k]
  std::vector<double> qref_h;  // host copy, [s]
  // solid sites and their new potentials (lbe_set_electrode_potential)
  std::vector<int> solid_h;
  int *solid_idx = nullptr;
  double *solid_val = nullptr;
  int nblk_charge = 0;
  double *qcur = nullptr;
  double *qhist = nullptr;
  int64_t qcap = 0, qlen = 0;

  // multigrid hierarchy (LBE_MG): level 0 is the lattice itself
  struct MgDev {
    MgLevel lv{};
    MgTransfer tr{};  // from the previous (finer) level
    uint32_t *mask = nullptr;
    bool own_mask = false;
    void *e = nullptr, *r = nullptr;  // correction and right-hand side (T)
    void *e2 = nullptr;               // second correction buffer (Jacobi smoothing)
    // host copies of the level's solid flags and fluid cells' systems (kept
    // for the small levels only: they decide the work-group split)
    std::vector<uint8_t> solid_h;
    std::vector<uint16_t> sys_h;
  };
  std::vector<MgDev> mg;
  int mg_coarse_sweeps = 0;
  int mg_nu1c = 0, mg_nu2c = 0;  // smoothing sweeps on the coarser levels
  double mg_jacobi = 0.0;   // > 0: Jacobi smoothing with this weight (else Gauss-Seidel)
  // coarsest level solved exactly: inverse of its operator over fluid cells
  int mg_nf = 0;
  void *mg_ainv = nullptr;  // T[nf * nf]
  int *mg_fcell = nullptr;  // fluid index -> cell
  // levels from mg_small_from down run in one work-group in LDS (-1: none)
  int mg_small_from = -1;
  MgSmall mg_small{};
  size_t mg_small_lds = 0;
  int *mg_groups = nullptr;  // range table of the independent groups (mg_small.ngroups > 1)

  // reverse mode: checkpoints kept by lbe_record, buffers of lbe_adjoint
  struct Tape {
    int64_t t0 = -1;      // step at which the recorded steps start (-1: none)
    int64_t nsteps = 0;
    int every = 1;        // steps between checkpoints
    int nck = 0;          // checkpoints at t0, t0 + every, ...; slot nck holds the end state
    int cap = 0;          // checkpoint slots allocated
    char *ck = nullptr;   // checkpoints: populations, concentrations, phi (and phi_prev)
    char *seg = nullptr;  // the recomputed states of one segment: rho, m, n, phi
    int seg_cap = 0;
    std::vector<int> hist;  // extrapolation history length at each checkpoint
  } tape;
  double *abar[2] = {nullptr, nullptr};  // adjoint of the pre-collision populations
  double *nbar[2] = {nullptr, nullptr};  // adjoint of the concentrations
  double *fbar = nullptr;      // adjoint of the force (3 N)
  double *adj_u = nullptr;     // velocity of the reverse step (3 N)
  double *lam = nullptr;       // last Poisson adjoint (warm start; zero on solid nodes)
  double *lam_sum = nullptr;   // Poisson adjoints summed over the reverse steps
  double *gphis = nullptr;     // gradient with respect to phi_s
  double *src_keep = nullptr;  // the forward Poisson source, restored after the sweep
  double *qbar_d = nullptr, *lb_acc = nullptr;
  uint8_t *type_d = nullptr;
  int adj_pred = 0;  // iterations the last adjoint solve needed

  // statistics
  int64_t step = 0;
  int last_iters = 0;
  double last_resid = 0.0;
  int64_t total_iters = 0;

  // profiling
  bool prof = false;
  struct Timed {
    hipEvent_t a, b;
    int64_t units;
  };
  std::vector<Timed> pending[KK_COUNT];
  std::vector<hipEvent_t> pool;
  double ms[KK_COUNT] = {};
  int64_t launches[KK_COUNT] = {};
  int64_t units[KK_COUNT] = {};

  std::string err;
};

namespace {

thread_local std::string g_init_error;

// An on/off switch from the environment: 1 for a value other than "0", 0
// for "0", dflt when unset or empty.
int env_flag(const char *name, int dflt) {
  const char *v = getenv(name);
  return v && *v ? (*v != '0' ? 1 : 0) : dflt;
}

int fail(lbe_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  else g_init_error = msg;
  return code;
}

int hip_fail(lbe_ctx *c, hipError_t e, const char *what) {
  return fail(c, e == hipErrorOutOfMemory ? LBE_ENOMEM : LBE_EDEVICE,
              std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

namespace lbe {
// A failure of a call without a context, reported by lbe_last_error(NULL).
int report_init_error(int code, const char *msg) { return fail(nullptr, code, msg); }
}  // namespace lbe

namespace {

#define HIPCHK(c, call)                                   \
  do {                                                    \
    hipError_t e_ = (call);                               \
    if (e_ != hipSuccess) return hip_fail((c), e_, #call); \
  } while (0)

// ---- profiling -----------------------------------------------------------

hipEvent_t take_event(lbe_ctx *c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

int flush_profile(lbe_ctx *c) {
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < KK_COUNT; ++k) {
    for (auto &pr : c->pending[k]) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, pr.a, pr.b) == hipSuccess) c->ms[k] += t;
      c->launches[k] += 1;
      c->units[k] += pr.units;
      c->pool.push_back(pr.a);
      c->pool.push_back(pr.b);
    }
    c->pending[k].clear();
  }
  return LBE_OK;
}

// Launches one kernel kind; `units` is the number of cells of the level it
// covers (lattice sites on the finest), summed per kind while profiling.
template <class Launch>
int run(lbe_ctx *c, KernelKind kind, int64_t units, Launch &&launch) {
  hipEvent_t a = nullptr, b = nullptr;
  if (c->prof) {
    a = take_event(c);
    b = take_event(c);
    if (a) (void)hipEventRecord(a, c->stream);
  }
  hipError_t e = launch();
  if (c->prof && a && b) {
    (void)hipEventRecord(b, c->stream);
    c->pending[kind].push_back({a, b, units});
    size_t tot = 0;
    for (int k = 0; k < KK_COUNT; ++k) tot += c->pending[k].size();
    if (tot > 16384) {
      int rc = flush_profile(c);
      if (rc) return rc;
    }
  }
  if (e != hipSuccess) return hip_fail(c, e, kKernelNames[kind]);
  return LBE_OK;
}

// ---- validation and geometry ---------------------------------------------

int validate(const lbe_params *p) {
  if (!p) return fail(nullptr, LBE_EINVAL, "params is NULL");
  if (p->nx < 1 || p->ny < 1 || p->nz < 1)
    return fail(nullptr, LBE_EINVAL, "lattice dimensions must be >= 1");
  // 32-bit site indices: 19 population arrays must stay below 2^31 entries
  if ((long long)p->nx * p->ny * p->nz > LBE_MAX_SITES)
    return fail(nullptr, LBE_EINVAL, "lattice larger than LBE_MAX_SITES");
  if (p->nspecies < 1 || p->nspecies > LBE_MAX_SPECIES)
    return fail(nullptr, LBE_EINVAL, "nspecies must be in 1..4");
  if (!(p->tau > 0.5)) return fail(nullptr, LBE_EINVAL, "tau must exceed 1/2");
  if (!(p->omega > 0.0 && p->omega < 2.0))
    return fail(nullptr, LBE_EINVAL, "omega must lie in (0, 2)");
  if (!(p->rho0 > 0.0) || !(p->lB >= 0.0) || !isfinite(p->lB) || !isfinite(p->rho0) ||
      !isfinite(p->tol) || p->max_iter < 0 || p->check_every < 1)
    return fail(nullptr, LBE_EINVAL, "bad rho0, lB, tol, max_iter or check_every");
  for (int k = 0; k < p->nspecies; ++k)
    if (!(p->D[k] >= 0.0) || !isfinite(p->D[k]))
      return fail(nullptr, LBE_EINVAL, "diffusion coefficients must be finite and >= 0");
  for (int a = 0; a < 3; ++a)
    if (!isfinite(p->Eapp[a])) return fail(nullptr, LBE_EINVAL, "applied field must be finite");
  if (p->flags & ~(LBE_ALLOW_FLOATING | LBE_EXTRAPOLATE | LBE_NAIVE_DIRICHLET | LBE_KRYLOV))
    return fail(nullptr, LBE_EINVAL, "unknown flags");
  if ((p->flags & LBE_KRYLOV) && p->poisson != LBE_MG)
    return fail(nullptr, LBE_EINVAL, "LBE_KRYLOV accelerates the multigrid solver only");
  if (p->precision != LBE_FP64 && p->precision != LBE_FP32_MIXED)
    return fail(nullptr, LBE_EINVAL, "unsupported precision form");
  if (p->poisson != LBE_SOR4 && p->poisson != LBE_MG)
    return fail(nullptr, LBE_EINVAL, "unsupported Poisson solver");
  if (p->poisson == LBE_MG && (p->mg_levels < 0 || p->mg_levels == 1 || p->mg_levels > 16 ||
                               p->mg_nu1 < 0 || p->mg_nu2 < 0 || p->mg_nu1 + p->mg_nu2 < 1 ||
                               p->mg_nu1_coarse < 0 || p->mg_nu2_coarse < 0))
    return fail(nullptr, LBE_EINVAL, "bad multigrid levels or smoothing counts");
  if (p->poisson == LBE_MG && p->mg_smoother != LBE_MG_JACOBI && p->mg_smoother != LBE_MG_GS4)
    return fail(nullptr, LBE_EINVAL, "unknown multigrid smoother");
  return LBE_OK;
}

struct HostGeometry {
  std::vector<uint32_t> mask;
  std::vector<int> iface;  // interface solid sites grouped by electrode
  std::vector<int> blk_elec, blk_begin, blk_end;
  uint32_t selfm = 0;
};

inline int wrap(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

int build_geometry(const lbe_params *p, const uint8_t *type, const uint16_t *sys, int ne,
                   HostGeometry &g) {
  const int nx = p->nx, ny = p->ny, nz = p->nz;
  const long N = (long)nx * ny * nz;
  for (int i = 1; i < NQ; ++i) {
    bool self = (CX[i] == 0 || nx == 1) && (CY[i] == 0 || ny == 1) && (CZ[i] == 0 || nz == 1);
    if (self) g.selfm |= 1u << (i - 1);
  }
  g.mask.assign(N, 0u);
  std::vector<int> nb((size_t)N * NQ);
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const long r = x + (long)nx * (y + (long)ny * z);
        uint32_t m = type[r] ? SOLID_BIT : (uint32_t)sys[r] << SYS_SHIFT;
        for (int i = 0; i < NQ; ++i) {
          const long rn = wrap(x + CX[i], nx) + (long)nx * (wrap(y + CY[i], ny) + (long)ny * wrap(z + CZ[i], nz));
          nb[(size_t)i * N + r] = (int)rn;
          if (i && type[rn]) m |= 1u << (i - 1);
          // independent systems: no fluid link may join two of them
          if (i && !type[r] && !type[rn] && sys[rn] != sys[r])
            return fail(nullptr, LBE_EGEOM, "a fluid link joins two systems");
        }
        g.mask[r] = m;
      }
  // four-colour order: neighbouring fluid nodes must differ in colour
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const long r = x + (long)nx * (y + (long)ny * z);
        if (type[r]) continue;
        const int cr = ((x + z) & 1) + 2 * ((y + z) & 1);
        for (int i = 1; i < NQ; ++i) {
          const int xn = wrap(x + CX[i], nx), yn = wrap(y + CY[i], ny), zn = wrap(z + CZ[i], nz);
          const long rn = nb[(size_t)i * N + r];
          if (rn == r || type[rn]) continue;
          if ((((xn + zn) & 1) + 2 * ((yn + zn) & 1)) == cr)
            return fail(nullptr, LBE_EGEOM,
                        "four-colour order invalid: periodic fluid extent along an axis is odd and > 2");
        }
      }
  // every fluid region must touch an electrode
  if (!(p->flags & LBE_ALLOW_FLOATING)) {
    std::vector<char> seen(N, 0);
    std::vector<long> stack;
    for (long r0 = 0; r0 < N; ++r0) {
      if (type[r0] || seen[r0]) continue;
      bool touches = false;
      stack.clear();
      stack.push_back(r0);
      seen[r0] = 1;
      while (!stack.empty()) {
        const long r = stack.back();
        stack.pop_back();
        for (int i = 1; i < NQ; ++i) {
          const long rn = nb[(size_t)i * N + r];
          if (type[rn]) {
            touches = true;
            continue;
          }
          if (!seen[rn]) {
            seen[rn] = 1;
            stack.push_back(rn);
          }
        }
      }
      if (!touches) return fail(nullptr, LBE_EGEOM, "a fluid region touches no electrode");
    }
  }
  // interface solid nodes per electrode and the charge kernel's block table
  constexpr int B = 256;
  std::vector<std::vector<int>> by_elec(ne + 1);
  for (long r = 0; r < N; ++r)
    if (type[r] && (g.mask[r] & ~SOLID_BIT) != ((1u << 18) - 1u)) by_elec[type[r]].push_back((int)r);
  for (int e = 1; e <= ne; ++e) {
    const int begin = (int)g.iface.size();
    g.iface.insert(g.iface.end(), by_elec[e].begin(), by_elec[e].end());
    const int end = (int)g.iface.size();
    for (int b = begin; b < end; b += B) {
      g.blk_elec.push_back(e - 1);
      g.blk_begin.push_back(b);
      g.blk_end.push_back(std::min(b + B, end));
    }
  }
  return LBE_OK;
}

template <class T>
int dalloc(lbe_ctx *c, T **ptr, size_t count) {
  if (count == 0) count = 1;
  HIPCHK(c, hipMalloc((void **)ptr, sizeof(T) * count));
  return LBE_OK;
}

// ---- steps ----------------------------------------------------------------

int read_scalars(lbe_ctx *c, int count) {
  HIPCHK(c, hipMemcpyAsync(c->hpin, c->dout, sizeof(double) * count, hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LBE_OK;
}

int reset_ctl(lbe_ctx *c) {
  // a new sequence number: whatever an earlier solve published is ignored
  // (its last stamp may still be on its way when this one starts)
  *c->ctl_h = SolveCtl{0.0, c->p.tol, 0, 0, 0, 0, 0, ++c->seq, 0ull, c->ctl_pub_d};
  c->checks_queued = 0;
  HIPCHK(c, hipMemcpyAsync(c->ctl, c->ctl_h, sizeof(SolveCtl), hipMemcpyHostToDevice, c->stream));
  return LBE_OK;
}

// The state of the running solve after every check queued so far: polled
// from the published copy (a check publishes when it ends, so the host learns
// the outcome without a stream synchronisation); if nothing is published for
// 100 ms, or there is no published copy, the block is copied back after a
// synchronisation instead (same result, slower).
int read_ctl(lbe_ctx *c) {
  if (c->ctl_pub) {
    volatile SolveCtl *v = c->ctl_pub;
    const auto t0 = std::chrono::steady_clock::now();
    for (long spin = 0;; ++spin) {
      const unsigned long long st = v->stamp;  // one 8-byte load
      const int done = (int)((st >> 31) & 1u), checks = (int)(st & 0x7fffffffu);
      if ((unsigned)(st >> 32) == (unsigned)c->seq && (done || checks >= c->checks_queued)) {
        // the values were written before the stamp (system-scope fence)
        c->ctl_h->done = done;
        c->ctl_h->checks = checks;
        c->ctl_h->resid = v->resid;
        c->ctl_h->count = v->count;
        c->ctl_h->iters = v->iters;
        c->ctl_h->nonfinite = v->nonfinite;
        return LBE_OK;
      }
      if ((spin & 1023) == 1023 &&
          std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(100))
        break;
    }
  }
  HIPCHK(c, hipMemcpyAsync(c->ctl_h, c->ctl, sizeof(SolveCtl), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LBE_OK;
}

// A warm-started iterative Poisson solve (Sec. II C) with device-side
// stopping.  step(m) queues m iterations (sweeps or cycles) and check(m) a
// residual check that counts those m; both are no-ops on the device once the
// solve is done.  Same schedule as the oracle: a check before the first
// iteration and after every `per_check`.  The host queues as many iterations
// as the previous time step needed and synchronises once; if that was not
// enough it adds a quarter more (at least one unit) and synchronises again.
// A unit (per_check iterations + check) is captured once as a HIP graph and
// replayed (not while per-kernel profiling is on).
int charges_to(lbe_ctx *c, double *dst, const SolveCtl *gate = nullptr);

template <class Step, class Check>
int run_solve(lbe_ctx *c, int per_check, bool learn, const char *unit, Step &&step,
              Check &&check) {
  const lbe_params &p = c->p;
  int rc;
  auto unit_direct = [&](int m) -> int {
    int r2 = step(m);
    return r2 ? r2 : check(m);
  };
  // every unit and the first check end in one residual check each
  auto unit_once = [&](int m) -> int {
    if (c->prof || !c->use_graphs || m != per_check) return unit_direct(m);
    if (!c->unit_exec) {
      hipGraph_t g = nullptr;
      HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
      const int r2 = unit_direct(m);
      const hipError_t e = hipStreamEndCapture(c->stream, &g);
      if (r2) {
        if (g) (void)hipGraphDestroy(g);
        return r2;
      }
      if (e != hipSuccess) return hip_fail(c, e, "graph capture");
      const hipError_t e2 = hipGraphInstantiate(&c->unit_exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e2 != hipSuccess) return hip_fail(c, e2, "graph instantiate");
    }
    HIPCHK(c, hipGraphLaunch(c->unit_exec, c->stream));
    return LBE_OK;
  };
  if (c->queue_units > 0) {
    // one step of a captured chunk: the control block cleared on the device,
    // the first check, a fixed number of units (each a no-op on the device
    // once the solve is done), the step's charge (of the converged
    // potential, or of the last iterate when the units did not suffice) and
    // its outcome; the host reads nothing
    HIPCHK(c, launch_ctl_reset(c->stream, c->ctl, p.tol));
    if ((rc = check(0))) return rc;
    for (int u = 0; u < c->queue_units; ++u)
      if ((rc = unit_direct(per_check))) return rc;
    if (c->charge_dst && (rc = charges_to(c, c->charge_dst, nullptr))) return rc;
    HIPCHK(c, launch_chunk_status(c->stream, c->ctl, c->chunk_st));
    return LBE_OK;
  }
  if ((rc = reset_ctl(c))) return rc;
  if (p.tol <= 0.0) {
    // exactly max_iter iterations on the schedule of a tolerance-driven
    // solve: a check before the first unit and one after each.  The checks
    // are part of the iteration where the solver needs them: the defect
    // correction's V-cycle and the mixed SOR sweeps take their right-hand
    // side (and the finest level's first sweep) from the check before them,
    // and the Krylov iteration starts from the first check's residual.  With
    // tol <= 0 no check ever ends the solve early.
    if ((rc = check(0))) return rc;
    c->checks_queued = 1;
    for (int it = 0; it < p.max_iter; it += per_check) {
      const int m = std::min(per_check, p.max_iter - it);
      if ((rc = unit_direct(m))) return rc;
      c->checks_queued += 1;
    }
    if ((rc = read_ctl(c))) return rc;
    c->last_iters = p.max_iter;
    c->last_resid = c->ctl_h->resid;
    c->total_iters += p.max_iter;
    if (c->ctl_h->nonfinite) return fail(c, LBE_ENONFINITE, "non-finite Poisson residual");
    return LBE_OK;
  }
  if ((rc = check(0))) return rc;
  c->checks_queued = 1;
  int queued = 0;
  // While profiling, one unit at a time with a read of the stop flag after
  // each, so that no timed launch is an early exit (the result is the same).
  int target = c->prof ? per_check : std::max(c->pred_iters, per_check);
  if (c->prof) {
    if ((rc = read_ctl(c))) return rc;
    if (c->ctl_h->done) target = 0;  // converged before the first unit
  }
  for (;;) {
    target = std::min(target, p.max_iter);
    while (queued < target) {
      const int m = std::min(per_check, p.max_iter - queued);
      if ((rc = unit_once(m))) return rc;
      c->checks_queued += 1;
      queued += m;
    }
    // the step's charge behind the queued units: it runs while the host
    // waits, and does nothing unless they reached the tolerance
    if (c->charge_dst && !c->prof) {
      if ((rc = charges_to(c, c->charge_dst, c->ctl))) return rc;
      c->charge_queued = true;
    }
    if ((rc = read_ctl(c))) return rc;
    if (c->ctl_h->done) break;
    // every check queued so far said not done, so the gated charge queued
    // behind them returned at once; it is queued again behind the next units
    c->charge_queued = false;
    if (queued >= p.max_iter) {
      c->last_iters = queued;
      c->last_resid = c->ctl_h->resid;
      c->total_iters += queued;
      char buf[160];
      snprintf(buf, sizeof buf, "Poisson not converged: residual %.3e after %d %s",
               c->ctl_h->resid, queued, unit);
      return fail(c, LBE_ENOCONV, buf);
    }
    target = queued + (c->prof ? per_check : std::max(per_check, queued / 4));
  }
  const int iters = c->ctl_h->iters;
  c->last_iters = iters;
  c->last_resid = c->ctl_h->resid;
  c->total_iters += iters;
  if (c->ctl_h->nonfinite) return fail(c, LBE_ENONFINITE, "non-finite Poisson residual");
  if (learn) c->pred_iters = iters;
  return LBE_OK;
}

// FP64 SOR on phi itself (Eq. 13 with Eq. 15, four colours).
int sor_solve(lbe_ctx *c, bool learn) {
  return run_solve(
      c, c->p.check_every, learn, "sweeps",
      [&](int m) -> int {
        for (int s2 = 0; s2 < m; ++s2)
          for (int col = 0; col < 4; ++col) {
            int rc = run(c, KK_SOR, c->L.n, [&] {
              return launch_sor_f64(c->stream, c->L, c->P, col, c->mask, c->src, c->phi, c->ctl);
            });
            if (rc) return rc;
          }
        return LBE_OK;
      },
      [&](int add) -> int {
        return run(c, KK_RESID, c->L.n, [&] {
          return launch_resid_f64(c->stream, c->L, c->mask, c->src, c->phi, c->partial, c->ctl,
                                  add);
        });
      });
}

// ---- multigrid hierarchy ----------------------------------------------------

// Four-colour order valid on a level: no two neighbouring fluid cells share a
// colour (self links excluded).
bool colouring_ok(int nx, int ny, int nz, const std::vector<uint8_t> &solid) {
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const long r = x + (long)nx * (y + (long)ny * z);
        if (solid[r]) continue;
        const int cr = ((x + z) & 1) + 2 * ((y + z) & 1);
        for (int i = 1; i < NQ; ++i) {
          const int xn = wrap(x + CX[i], nx), yn = wrap(y + CY[i], ny), zn = wrap(z + CZ[i], nz);
          const long rn = xn + (long)nx * (yn + (long)ny * zn);
          if (rn == r || solid[rn]) continue;
          if ((((xn + zn) & 1) + 2 * ((yn + zn) & 1)) == cr) return false;
        }
      }
  return true;
}

std::vector<uint32_t> level_mask(int nx, int ny, int nz, const std::vector<uint8_t> &solid) {
  std::vector<uint32_t> m((size_t)nx * ny * nz);
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const long r = x + (long)nx * (y + (long)ny * z);
        uint32_t v = solid[r] ? SOLID_BIT : 0u;
        for (int i = 1; i < NQ; ++i) {
          const long rn = wrap(x + CX[i], nx) + (long)nx * (wrap(y + CY[i], ny) + (long)ny * wrap(z + CZ[i], nz));
          if (solid[rn]) v |= 1u << (i - 1);
        }
        m[r] = v;
      }
  return m;
}

uint32_t level_selfm(int nx, int ny, int nz) {
  uint32_t s = 0;
  for (int i = 1; i < NQ; ++i)
    if ((CX[i] == 0 || nx == 1) && (CY[i] == 0 || ny == 1) && (CZ[i] == 0 || nz == 1))
      s |= 1u << (i - 1);
  return s;
}

// Coarsen one level: cells pair up along every axis longer than 1 (one half
// block at the end of an odd axis); offsets minimise blocks that mix solid
// and fluid; a block is solid when at least half of its children are, or
// when its fluid children belong to different independent systems (so that
// batched systems stay decoupled on every level).  sys / csys: system of
// each fluid cell of the fine / coarse level.
void coarsen(int nx, int ny, int nz, const std::vector<uint8_t> &solid,
             const std::vector<uint16_t> &sys, int &cx, int &cy, int &cz, int &ox, int &oy,
             int &oz, std::vector<uint8_t> &csolid, std::vector<uint16_t> &csys) {
  cx = nx > 1 ? (nx + 1) / 2 : 1;
  cy = ny > 1 ? (ny + 1) / 2 : 1;
  cz = nz > 1 ? (nz + 1) / 2 : 1;
  const long nc = (long)cx * cy * cz;
  long best = -1;
  std::vector<int> ns(nc), nf(nc);
  for (int tz = 0; tz < (nz > 1 ? 2 : 1); ++tz)
    for (int ty = 0; ty < (ny > 1 ? 2 : 1); ++ty)
      for (int tx = 0; tx < (nx > 1 ? 2 : 1); ++tx) {
        std::fill(ns.begin(), ns.end(), 0);
        std::fill(nf.begin(), nf.end(), 0);
        for (int z = 0; z < nz; ++z)
          for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
              const long r = x + (long)nx * (y + (long)ny * z);
              const long R = (wrap(x - tx, nx) / 2) + (long)cx * ((wrap(y - ty, ny) / 2) + (long)cy * (wrap(z - tz, nz) / 2));
              (solid[r] ? ns : nf)[R]++;
            }
        long mixed = 0;
        for (long R = 0; R < nc; ++R) mixed += (ns[R] && nf[R]);
        if (best < 0 || mixed < best) {
          best = mixed;
          ox = tx;
          oy = ty;
          oz = tz;
          csolid.assign(nc, 0);
          for (long R = 0; R < nc; ++R) csolid[R] = 2 * ns[R] >= ns[R] + nf[R];
        }
      }
  // systems of the coarse cells, with the chosen offsets
  csys.assign(nc, 0);
  std::vector<uint8_t> seen(nc, 0);
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const long r = x + (long)nx * (y + (long)ny * z);
        if (solid[r]) continue;
        const long R = (wrap(x - ox, nx) / 2) + (long)cx * ((wrap(y - oy, ny) / 2) + (long)cy * (wrap(z - oz, nz) / 2));
        if (!seen[R]) {
          seen[R] = 1;
          csys[R] = sys[r];
        } else if (csys[R] != sys[r]) {
          csolid[R] = 1;
        }
      }
}

// Dense inverse of the coarsest operator A e = (6/h^2) sum_i w_i s_i (e - e_i)
// over its fluid cells (Cholesky in FP64; A is symmetric positive definite when
// every fluid region touches an electrode).  Not built when the level has
// more than MG_MAX_DENSE fluid cells or A is singular (floating regions): the
// coarsest level is then swept instead.

int build_coarse_inverse(lbe_ctx *c, const std::vector<uint8_t> &solid) {
  const MgLevel &lv = c->mg.back().lv;
  std::vector<int> fidx(lv.n, -1), fcell;
  for (int r = 0; r < lv.n; ++r)
    if (!solid[r]) {
      fidx[r] = (int)fcell.size();
      fcell.push_back(r);
    }
  const int nf = (int)fcell.size();
  if (nf == 0 || nf > MG_MAX_DENSE) return LBE_OK;
  std::vector<double> A((size_t)nf * nf, 0.0);
  const double sc = 6.0 * lv.inv_h2;
  for (int j = 0; j < nf; ++j) {
    const int r = fcell[j];
    const int z = r / lv.nxy, y = (r - z * lv.nxy) / lv.nx, x = r - z * lv.nxy - y * lv.nx;
    for (int i = 1; i < NQ; ++i) {
      if ((lv.selfm >> (i - 1)) & 1u) continue;
      const int rn = wrap(x + CX[i], lv.nx) + lv.nx * (wrap(y + CY[i], lv.ny) + lv.ny * wrap(z + CZ[i], lv.nz));
      if (solid[rn]) {
        A[(size_t)j * nf + j] += sc * lv.wall * WQ[i];
      } else {
        A[(size_t)j * nf + j] += sc * WQ[i];
        A[(size_t)j * nf + fidx[rn]] -= sc * WQ[i];
      }
    }
  }
  // Cholesky A = L L^T (lower triangle in place)
  for (int j = 0; j < nf; ++j) {
    double d = A[(size_t)j * nf + j];
    for (int k = 0; k < j; ++k) d -= A[(size_t)j * nf + k] * A[(size_t)j * nf + k];
    if (!(d > 1e-12 * sc)) return LBE_OK;  // singular: keep the sweeps
    d = sqrt(d);
    A[(size_t)j * nf + j] = d;
    for (int i = j + 1; i < nf; ++i) {
      double v = A[(size_t)i * nf + j];
      for (int k = 0; k < j; ++k) v -= A[(size_t)i * nf + k] * A[(size_t)j * nf + k];
      A[(size_t)i * nf + j] = v / d;
    }
  }
  // inverse column by column: solve L y = e_k, L^T x = y
  std::vector<double> inv((size_t)nf * nf), y(nf);
  for (int col = 0; col < nf; ++col) {
    for (int i = 0; i < nf; ++i) {
      double v = (i == col) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) v -= A[(size_t)i * nf + k] * y[k];
      y[i] = v / A[(size_t)i * nf + i];
    }
    for (int i = nf - 1; i >= 0; --i) {
      double v = y[i];
      for (int k = i + 1; k < nf; ++k) v -= A[(size_t)k * nf + i] * inv[(size_t)k * nf + col];
      inv[(size_t)i * nf + col] = v / A[(size_t)i * nf + i];
    }
  }
  // the kernels read the inverse column-major: at[j * nf + row] = inv[row][j]
  std::vector<double> at((size_t)nf * nf);
  for (int row = 0; row < nf; ++row)
    for (int j = 0; j < nf; ++j) at[(size_t)j * nf + row] = inv[(size_t)row * nf + j];
  inv.swap(at);
  HIPCHK(c, hipMalloc((void **)&c->mg_fcell, sizeof(int) * nf));
  HIPCHK(c, hipMemcpy(c->mg_fcell, fcell.data(), sizeof(int) * nf, hipMemcpyHostToDevice));
  if (c->mixed) {
    std::vector<float> f32(inv.begin(), inv.end());
    HIPCHK(c, hipMalloc(&c->mg_ainv, sizeof(float) * f32.size()));
    HIPCHK(c, hipMemcpy(c->mg_ainv, f32.data(), sizeof(float) * f32.size(), hipMemcpyHostToDevice));
  } else {
    HIPCHK(c, hipMalloc(&c->mg_ainv, sizeof(double) * inv.size()));
    HIPCHK(c, hipMemcpy(c->mg_ainv, inv.data(), sizeof(double) * inv.size(), hipMemcpyHostToDevice));
  }
  c->mg_nf = nf;
  return LBE_OK;
}

// Independent groups of the small levels (batched systems): when, on every
// level the one-work-group kernel handles, the fluid cells of each system lie
// in a cyclic index range of their own (the ranges may wrap through the
// periodic boundary), no fluid cell has a fluid cell of another system among
// its 26 neighbours (so neither the stencil nor the prolongation couples two
// systems, and the exact coarsest solve is block-diagonal by system), each
// system's part of the V-cycle is computed by a work-group of its own, all in
// one launch.  The ranges are widened over the solid cells after them so
// that they tile every level.  The table holds, per level and group, the
// first cell and the length of its range, and for the exact solve the first
// fluid row and the row count.  The arithmetic of every cell is that of one
// work-group doing everything (the exact solve skips only columns that are
// exact zeros), so the results are the same bit for bit.
int plan_small_groups(lbe_ctx *c) {
  MgSmall &S = c->mg_small;
  S.ngroups = 1;
  S.groups = nullptr;
  {
    const char *ng = getenv("LBE_NO_SMALL_GROUPS");  // one work-group (same results)
    if (ng && *ng && *ng != '0') return LBE_OK;
  }
  const int k0 = c->mg_small_from, L = (int)c->mg.size();
  for (int k = k0; k < L; ++k)
    if (c->mg[k].solid_h.size() != (size_t)c->mg[k].lv.n) return LBE_OK;
  // systems present on the first small level
  const lbe_ctx::MgDev &F = c->mg[k0];
  std::vector<int> gid(LBE_MAX_SYSTEMS, -1);
  int G = 0;
  for (int r = 0; r < F.lv.n; ++r)
    if (!F.solid_h[r] && gid[F.sys_h[r]] < 0) gid[F.sys_h[r]] = G++;
  if (G < 2) return LBE_OK;
  // per level and group: first cell and length; then the exact solve's rows
  std::vector<int> table((size_t)(S.nlev + 1) * G * 2, 0);
  for (int k = k0; k < L; ++k) {
    const lbe_ctx::MgDev &D = c->mg[k];
    const MgLevel &lv = D.lv;
    const int n = lv.n;
    std::vector<std::vector<int>> cells(G);
    for (int r = 0; r < n; ++r) {
      if (D.solid_h[r]) continue;
      const int g = gid[D.sys_h[r]];
      if (g < 0) return LBE_OK;
      cells[g].push_back(r);
      const int z = r / lv.nxy, y = (r - z * lv.nxy) / lv.nx, x = r - z * lv.nxy - y * lv.nx;
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            const int rn = wrap(x + dx, lv.nx) + lv.nx * (wrap(y + dy, lv.ny) + lv.ny * wrap(z + dz, lv.nz));
            if (!D.solid_h[rn] && D.sys_h[rn] != D.sys_h[r]) return LBE_OK;
          }
    }
    // each group's smallest cyclic interval: the complement of the largest
    // gap between its cells
    std::vector<int> owner(n, -1), st(G, -1);
    std::vector<std::pair<int, int>> starts;
    for (int g = 0; g < G; ++g) {
      const std::vector<int> &v = cells[g];
      if (v.empty()) continue;
      const int m = (int)v.size();
      int best = 0, gap = v[0] + n - v[m - 1];
      for (int i = 0; i + 1 < m; ++i)
        if (v[i + 1] - v[i] > gap) {
          gap = v[i + 1] - v[i];
          best = i + 1;
        }
      const int s0 = v[best], len = n - gap + 1;
      for (int i = 0; i < len; ++i) {
        const int r = (s0 + i) % n;
        if (owner[r] >= 0) return LBE_OK;  // two systems interleave
        owner[r] = g;
      }
      st[g] = s0;
      starts.push_back({s0, g});
    }
    // widen each range up to the next one (cyclically), so that they tile
    std::sort(starts.begin(), starts.end());
    int *row = table.data() + (size_t)(k - k0) * G * 2;
    const int np = (int)starts.size();
    for (int i = 0; i < np; ++i) {
      const int s0 = starts[i].first, g = starts[i].second;
      const int s1 = starts[(i + 1) % np].first;
      row[2 * g] = s0;
      row[2 * g + 1] = np == 1 ? n : ((s1 - s0) % n + n) % n;
    }
    (void)st;
  }
  // the exact solve's rows: the fluid cells of the coarsest level in each
  // group's range, a cyclic range of fluid indices (fluid cells in cell order)
  if (S.ainv) {
    const lbe_ctx::MgDev &D = c->mg[L - 1];
    const int n = D.lv.n;
    std::vector<int> fidx(n, -1);
    int nf = 0;
    for (int r = 0; r < n; ++r)
      if (!D.solid_h[r]) fidx[r] = nf++;
    if (nf != S.nf) return LBE_OK;
    const int *crow = table.data() + (size_t)(S.nlev - 1) * G * 2;
    int *frow = table.data() + (size_t)S.nlev * G * 2;
    for (int g = 0; g < G; ++g) {
      int f0 = -1, cnt = 0;
      for (int i = 0; i < crow[2 * g + 1]; ++i) {
        const int r = (crow[2 * g] + i) % n;
        if (fidx[r] < 0) continue;
        if (f0 < 0) f0 = fidx[r];
        ++cnt;
      }
      frow[2 * g] = f0 < 0 ? 0 : f0;
      frow[2 * g + 1] = cnt;
    }
  }
  HIPCHK(c, hipMalloc((void **)&c->mg_groups, sizeof(int) * table.size()));
  HIPCHK(c, hipMemcpy(c->mg_groups, table.data(), sizeof(int) * table.size(),
                      hipMemcpyHostToDevice));
  S.ngroups = G;
  S.groups = c->mg_groups;
  return LBE_OK;
}

// Choose the first level, of at most 2048 cells, from which the rest of the
// hierarchy fits in one work-group's LDS (correction and right-hand side per
// cell in T, flag words).  Larger levels are faster as multi-block kernels.
int plan_small_levels(lbe_ctx *c) {
  c->mg_small_from = -1;
  if (c->mg.size() < 2 || getenv("LBE_NO_SMALL_MG")) return LBE_OK;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) return LBE_OK;
  const size_t limit = prop.sharedMemPerBlock;
  const size_t tsz = c->mixed ? sizeof(float) : sizeof(double);
  const int L = (int)c->mg.size();
  for (int from = 0; from < L; ++from) {
    // one compute unit sweeps the set: only worth it while the levels are tiny
    if (L - from > MG_MAX_SMALL || c->mg[from].lv.n > 2048) continue;
    // per cell: correction and right-hand side (and the second Jacobi buffer)
    const size_t per_cell = c->mg_jacobi > 0.0 ? 3 : 2;
    // the exact coarsest solve's compact right-hand side and its part sums
    const size_t dense = c->mg_nf > 0 ? (size_t)c->mg_nf + 1024 : 0;
    size_t tbytes = tsz * dense, mbytes = 0;
    for (int k = from; k < L; ++k) {
      tbytes += per_cell * tsz * (size_t)c->mg[k].lv.n;
      mbytes += 4 * (size_t)c->mg[k].lv.n;
    }
    const size_t total = tbytes + mbytes;
    if (total > limit) continue;
    MgSmall S{};
    S.nlev = L - from;
    size_t te = 0;  // in T elements
    for (int k = 0; k < S.nlev; ++k) {
      const lbe_ctx::MgDev &D = c->mg[from + k];
      S.lv[k] = D.lv;
      if (k) S.tr[k] = D.tr;
      S.mask[k] = D.mask;
      S.off_e[k] = (int)te;
      te += D.lv.n;
      S.off_r[k] = (int)te;
      te += D.lv.n;
      S.off_e2[k] = (int)te;
      if (per_cell == 3) te += D.lv.n;
    }
    S.off_x = (int)te;
    te += dense;
    size_t me = te * tsz / 4;  // flag words follow, in 4-byte units
    for (int k = 0; k < S.nlev; ++k) {
      S.off_m[k] = (int)me;
      me += c->mg[from + k].lv.n;
    }
    S.nu1 = c->mg_nu1c;
    S.nu2 = c->mg_nu2c;
    S.nf = c->mg_nf;
    S.ainv = c->mg_ainv;
    S.fcell = c->mg_fcell;
    S.coarse_sweeps = c->mg_coarse_sweeps;
    S.omega = c->p.omega;
    S.jacobi = c->mg_jacobi;
    const hipError_t e = c->mixed ? prepare_mg_small<float>(total) : prepare_mg_small<double>(total);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return LBE_OK;
    }
    c->mg_small = S;
    c->mg_small_from = from;
    c->mg_small_lds = total;
    return plan_small_groups(c);
  }
  return LBE_OK;
}

int build_multigrid(lbe_ctx *c, const uint8_t *type, bool only_top) {
  const size_t esz = c->mixed ? sizeof(float) : sizeof(double);
  const int maxl = only_top ? 1 : (c->p.mg_levels > 0 ? c->p.mg_levels : 16);
  int nx = c->p.nx, ny = c->p.ny, nz = c->p.nz;
  std::vector<uint8_t> solid((size_t)nx * ny * nz);
  for (size_t r = 0; r < solid.size(); ++r) solid[r] = type[r] != 0;
  std::vector<uint16_t> sys = c->sys_h;
  lbe_ctx::MgDev l0;
  l0.lv = make_level(nx, ny, nz, c->L.selfm, 1.0, c->L.wall, c->L.xcd);
  l0.mask = c->mask;
  if (l0.lv.n <= MG_GROUP_SCAN) {
    l0.solid_h = solid;
    l0.sys_h = sys.empty() ? std::vector<uint16_t>(solid.size(), 0) : sys;
  }
  HIPCHK(c, hipMalloc(&l0.e, esz * l0.lv.n));
  HIPCHK(c, hipMalloc(&l0.e2, esz * l0.lv.n));
  HIPCHK(c, hipMalloc(&l0.r, esz * l0.lv.n));
  c->mg.push_back(l0);
  double h2 = 1.0;
  for (int l = 1; l < maxl; ++l) {
    if (c->p.mg_levels == 0 && (long)nx * ny * nz <= MG_MAX_DENSE) break;
    if (nx <= 2 && ny <= 2 && nz <= 2) break;
    int cx, cy, cz, ox = 0, oy = 0, oz = 0;
    std::vector<uint8_t> cs;
    std::vector<uint16_t> csy;
    coarsen(nx, ny, nz, solid, sys, cx, cy, cz, ox, oy, oz, cs, csy);
    if (std::find(cs.begin(), cs.end(), 0) == cs.end()) break;  // no fluid left
    // the four-colour smoother needs a proper colouring on every level;
    // Jacobi smoothing (and the dense coarsest solve) does not
    if (c->mg_jacobi == 0.0 && !colouring_ok(cx, cy, cz, cs)) break;
    h2 *= 4.0;
    lbe_ctx::MgDev L;
    L.lv = make_level(cx, cy, cz, level_selfm(cx, cy, cz), h2, c->L.wall, c->L.xcd);
    L.tr = MgTransfer{c->mg.back().lv, L.lv, ox, oy, oz};
    const std::vector<uint32_t> m = level_mask(cx, cy, cz, cs);
    HIPCHK(c, hipMalloc((void **)&L.mask, sizeof(uint32_t) * m.size()));
    L.own_mask = true;
    c->mg.push_back(L);  // owned from here on, freed with the context
    lbe_ctx::MgDev &B = c->mg.back();
    if (B.lv.n <= MG_GROUP_SCAN) {
      B.solid_h = cs;
      B.sys_h = csy;
    }
    HIPCHK(c, hipMemcpy(B.mask, m.data(), sizeof(uint32_t) * m.size(), hipMemcpyHostToDevice));
    HIPCHK(c, hipMalloc(&B.e, esz * B.lv.n));
    HIPCHK(c, hipMalloc(&B.e2, esz * B.lv.n));
    HIPCHK(c, hipMalloc(&B.r, esz * B.lv.n));
    HIPCHK(c, hipMemset(B.e, 0, esz * B.lv.n));
    nx = cx;
    ny = cy;
    nz = cz;
    solid.swap(cs);
    sys.swap(csy);
  }
  const MgLevel &top = c->mg.back().lv;
  c->mg_coarse_sweeps = 2 * std::max({top.nx, top.ny, top.nz}) + 10;
  // the coarsest level (the only one on a lattice of at most 512 cells) is
  // inverted exactly when it is small and non-singular
  if (!only_top) {
    int rc = build_coarse_inverse(c, solid);
    if (rc) return rc;
  }
  return plan_small_levels(c);
}

// One V-cycle from level l: e (zeroed by the residual / restriction kernel)
// -> pre-smoothing -> restriction -> V-cycle below -> prolongation ->
// post-smoothing; *out receives the level's correction.
// One V-cycle on level l for A e = r (e starts at 0); *out receives the
// buffer holding e.  With phi_add (finest level), the last smoothing launch
// also adds e to phi and *added is set; otherwise the caller adds it.
template <class T>
int mg_vcycle(lbe_ctx *c, size_t l, T **out, double *phi_add = nullptr, bool *added = nullptr,
              bool first_done = false) {
  lbe_ctx::MgDev &L = c->mg[l];
  T *A = (T *)L.e, *r = (T *)L.r;
  int rc;
  if ((int)l == c->mg_small_from) {
    *out = A;
    return run(c, KK_MG_SMALL, L.lv.n, [&] {
      return launch_mg_small<T>(c->stream, c->mg_small, c->mg_small_lds, r, A, c->ctl);
    });
  }
  if (l + 1 == c->mg.size()) {
    *out = A;
    if (c->mg_ainv)
      return run(c, KK_MG_COARSE, L.lv.n, [&] {
        return launch_mg_coarse_dense<T>(c->stream, c->mg_nf, (const T *)c->mg_ainv, c->mg_fcell,
                                         r, A, c->ctl);
      });
    return run(c, KK_MG_COARSE, L.lv.n, [&] {
      return launch_mg_coarse<T>(c->stream, L.lv, c->p.omega, c->mg_jacobi, c->mg_coarse_sweeps,
                                 L.mask, r, A, (T *)L.e2, c->ctl);
    });
  }
  const KernelKind sk = l == 0 ? KK_MG_SMOOTH0 : KK_MG_SMOOTH;
  T *cur = A, *alt = (T *)L.e2;
  const int nu1 = l == 0 ? c->p.mg_nu1 : c->mg_nu1c, nu2 = l == 0 ? c->p.mg_nu2 : c->mg_nu2c;
  // four-colour Gauss-Seidel in place, or damped Jacobi from cur into the
  // other buffer, which then becomes cur; the last sweep on the finest level
  // may add the result to phi
  auto smooth = [&](int sweeps, double *add_to) -> int {
    if (c->mg_jacobi > 0.0) {
      for (int s2 = 0; s2 < sweeps; ++s2) {
        const bool last = s2 + 1 == sweeps;
        const KernelKind kind = last && add_to ? KK_MG_SMOOTH0_PHI : sk;
        const int r2 = run(c, kind, L.lv.n, [&] {
          return launch_jacobi<T>(c->stream, L.lv, c->mg_jacobi, L.lv.h2 / 6.0, L.mask, r, cur,
                                  alt, c->ctl, last ? add_to : nullptr, c->rings);
        });
        if (r2) return r2;
        std::swap(cur, alt);
      }
      return LBE_OK;
    }
    for (int s2 = 0; s2 < sweeps; ++s2)
      for (int col = 0; col < 4; ++col) {
        const int r2 = run(c, sk, L.lv.n, [&] {
          return launch_mg_smooth<T>(c->stream, L.lv, 1.0, col, L.mask, r, cur, c->ctl);
        });
        if (r2) return r2;
      }
    return LBE_OK;
  };
  // with first_done the correction already holds its first Jacobi sweep
  if ((rc = smooth(first_done ? nu1 - 1 : nu1, nullptr))) return rc;
  lbe_ctx::MgDev &C = c->mg[l + 1];
  // when the level below is smoothed by the global Jacobi kernels, its first
  // sweep starts from zero and is pointwise: the restriction writes it
  const bool start = c->coarse_start && c->mg_jacobi > 0.0 && c->mg_nu1c >= 1 &&
                     (int)(l + 1) != c->mg_small_from && l + 2 < c->mg.size();
  rc = run(c, KK_MG_RESTRICT, L.lv.n, [&] {
    return launch_mg_restrict<T>(c->stream, C.tr, L.mask, C.mask, r, cur, (T *)C.r, (T *)C.e,
                                 c->ctl, c->tiles, start ? c->mg_jacobi : 0.0, C.lv.h2 / 6.0,
                                 c->rings);
  });
  if (rc) return rc;
  T *ce = nullptr;
  if ((rc = mg_vcycle<T>(c, l + 1, &ce, nullptr, nullptr, start))) return rc;
  rc = run(c, KK_MG_PROLONG, L.lv.n, [&] {
    return launch_mg_prolong<T>(c->stream, C.tr, L.mask, C.mask, (const T *)ce, cur, c->ctl,
                                c->rings);
  });
  if (rc) return rc;
  if ((rc = smooth(nu2, phi_add))) return rc;
  if (added) *added = c->mg_jacobi > 0.0 && nu2 > 0 && phi_add != nullptr;
  *out = cur;
  return LBE_OK;
}

// Defect correction: residual in FP64 (which also zeroes e and stores the
// right-hand side for the correction), one V-cycle for e, phi += e.  With
// LBE_KRYLOV the V-cycle preconditions flexible conjugate gradients instead
// (one V-cycle and one operator application per iteration).
template <class T>
int mg_solve(lbe_ctx *c, bool learn) {
  lbe_ctx::MgDev &L0 = c->mg[0];
  // the kernel that writes the finest level's right-hand side (the residual
  // check, or the Krylov update) takes the V-cycle's first Jacobi sweep
  // (from 0) when that level is smoothed by the global kernels
  const double first_sweep = (c->mg_jacobi > 0.0 && c->p.mg_nu1 >= 1 && c->mg.size() > 1 &&
                              c->mg_small_from != 0 && c->coarse_start)
                                 ? c->mg_jacobi
                                 : 0.0;
  if (c->kc) {
    const int n = L0.lv.n;
    return run_solve(
        c, 1, learn, "cycles",
        [&](int m) -> int {
          for (int k = 0; k < m; ++k) {
            T *z = nullptr;
            int rc = mg_vcycle<T>(c, 0, &z, nullptr, nullptr, first_sweep > 0.0);
            if (rc) return rc;
            rc = run(c, KK_FCG_APPLY, n, [&] {
              return launch_fcg_apply<T>(c->stream, L0.lv, c->mask, (const T *)z,
                                         (const T *)c->kq, (const T *)c->kp,
                                         c->kr, c->kaz, c->partial, c->kc, c->ctl, c->rings);
            });
            if (rc) return rc;
            // every iteration ends with its own stop check (one cycle each)
            rc = run(c, KK_FCG_UPDATE, n, [&] {
              return launch_fcg_update<T>(c->stream, n, c->mask, (const T *)z, c->kaz,
                                          (T *)c->kp, (T *)c->kq, c->phi, c->kr, (T *)L0.r,
                                          (T *)L0.e, c->partial, c->kc, c->ctl, 1, L0.lv,
                                          first_sweep);
            });
            if (rc) return rc;
          }
          return LBE_OK;
        },
        [&](int add) -> int {
          if (add) return LBE_OK;  // each update kernel has checked already
          return run(c, KK_MG_RESID, n, [&] {
            return launch_mg_outer_resid<T>(c->stream, L0.lv, c->mask, c->src, c->phi,
                                            (T *)L0.r, (T *)L0.e, c->partial, c->ctl, 0, c->kr,
                                            c->kc, first_sweep, c->rings);
          });
        });
  }
  return run_solve(
      c, 1, learn, "cycles",
      [&](int m) -> int {
        for (int k = 0; k < m; ++k) {
          T *e0 = nullptr;
          bool added = false;
          int rc = mg_vcycle<T>(c, 0, &e0, c->phi, &added, first_sweep > 0.0);
          if (rc) return rc;
          if (added) continue;  // the last smoothing launch has corrected phi
          rc = run(c, KK_CORRECT, L0.lv.n, [&] {
            return launch_mg_correct<T>(c->stream, L0.lv.n, c->mask, (const T *)e0, c->phi,
                                        c->ctl);
          });
          if (rc) return rc;
        }
        return LBE_OK;
      },
      [&](int add) -> int {
        return run(c, KK_MG_RESID, L0.lv.n, [&] {
          return launch_mg_outer_resid<T>(c->stream, L0.lv, c->mask, c->src, c->phi, (T *)L0.r,
                                          (T *)L0.e, c->partial, c->ctl, add, nullptr, nullptr,
                                          first_sweep, c->rings);
        });
      });
}

// room for `rows` charge rows in all (default: one more than recorded)
int grow_history(lbe_ctx *c, int64_t rows = -1) {
  if (rows < 0) rows = c->qlen + 1;
  if (rows <= c->qcap) return LBE_OK;
  int64_t cap = c->qcap ? 2 * c->qcap : 4096;
  while (cap < rows) cap *= 2;
  double *nh = nullptr;
  int rc = dalloc(c, &nh, (size_t)cap * std::max(c->ne, 1));
  if (rc) return rc;
  if (c->qhist) {
    HIPCHK(c, hipMemcpyAsync(nh, c->qhist, sizeof(double) * c->qlen * std::max(c->ne, 1),
                             hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    (void)hipFree(c->qhist);
  }
  c->qhist = nh;
  c->qcap = cap;
  return LBE_OK;
}

// Mixed form with SOR: FP64 residual, check_every FP32 SOR sweeps on the
// correction from zero (the same iterates as SOR on phi, accumulated in FP32),
// then phi += e.  Counts sweeps.
int mixed_sor_solve(lbe_ctx *c, bool learn) {
  lbe_ctx::MgDev &L0 = c->mg[0];
  return run_solve(
      c, c->p.check_every, learn, "sweeps",
      [&](int m) -> int {
        for (int s2 = 0; s2 < m; ++s2)
          for (int col = 0; col < 4; ++col) {
            int rc = run(c, KK_SOR32, L0.lv.n, [&] {
              return launch_mg_smooth<float>(c->stream, L0.lv, c->p.omega, col, c->mask,
                                             (const float *)L0.r, (float *)L0.e, c->ctl);
            });
            if (rc) return rc;
          }
        return run(c, KK_CORRECT, L0.lv.n, [&] {
          return launch_mg_correct<float>(c->stream, L0.lv.n, c->mask, (const float *)L0.e,
                                          c->phi, c->ctl);
        });
      },
      [&](int add) -> int {
        return run(c, KK_MG_RESID, L0.lv.n, [&] {
          return launch_mg_outer_resid<float>(c->stream, L0.lv, c->mask, c->src, c->phi,
                                              (float *)L0.r, (float *)L0.e, c->partial, c->ctl,
                                              add, nullptr, nullptr, 0.0, c->rings);
        });
      });
}

// learn: remember the iteration count to size the next time step's queue
int poisson_solve(lbe_ctx *c, bool learn) {
  if (c->mixed) return c->p.poisson == LBE_MG ? mg_solve<float>(c, learn) : mixed_sor_solve(c, learn);
  if (c->p.poisson == LBE_MG) return mg_solve<double>(c, learn);
  return sor_solve(c, learn);
}

int charges_to(lbe_ctx *c, double *dst, const SolveCtl *gate) {
  if (c->ne == 0) return LBE_OK;
  if (c->nblk_charge == 0) {  // no electrode touches the fluid
    HIPCHK(c, hipMemsetAsync(dst, 0, sizeof(double) * c->ne, c->stream));
    return LBE_OK;
  }
  const double q_scale = -6.0 / (4.0 * M_PI * c->p.lB);
  return run(c, KK_CHARGE, c->L.n, [&] {
    return launch_charge(c->stream, c->L, q_scale, c->mask, c->phi, c->iface, c->blk_elec,
                         c->blk_begin, c->blk_end, c->nblk_charge, c->ne, c->partial,
                         dst, gate);
  });
}

int record_charge(lbe_ctx *c) {
  int rc = grow_history(c);
  if (rc) return rc;
  rc = charges_to(c, c->qhist + c->qlen * std::max(c->ne, 1));
  if (rc) return rc;
  c->qlen++;
  return LBE_OK;
}

// Back to the start of a step whose Poisson solve failed: n(t) and f(t) are
// still in the buffers the step read, phi(t) in the copy pass B made (the
// extrapolation history, else phi_keep).  Of the history only phi(t-2) is
// lost, so the retried step starts from a linear extrapolation.
int rewind_step(lbe_ctx *c, int a, int hist, bool record) {
  c->cur = a;
  if (record) c->step--;
  double *keep = c->phi_prev ? c->phi_prev : c->phi_keep;
  const int shift = c->phi_prev ? 1 : 0;
  int rc = run(c, KK_REWIND, c->L.n, [&] {
    if (c->mixed)
      return launch_rewind_f32(c->stream, c->L, c->P, c->mask, c->nu32[a], c->lo32[a], c->src,
                               c->phi, keep, shift);
    return launch_rewind_f64(c->stream, c->L, c->P, c->mask, c->n[a], c->src, c->phi, keep, shift);
  });
  if (rc) return rc;
  if (c->phi_prev) c->extrap_hist = std::min(hist, 1);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LBE_OK;
}

// record = false: a replay of a recorded step (reverse mode), which neither
// counts the step nor appends its charge
// The two passes of a step from buffers a to b: LB and ion link fluxes
// (pass A), advection and the new concentrations (pass B), which also moves
// phi to the start of the step's solve.  hist: the extrapolation history.
int step_passes(lbe_ctx *c, int a, int b, int hist) {
  // pass B keeps phi(t) for a rewind: in the extrapolation history, else in
  // phi_keep (order -1: a plain copy)
  double *keep = c->phi_prev ? c->phi_prev : c->phi_keep;
  const int order = c->phi_prev ? hist : -1;
  int rc = run(c, KK_FLUID, c->L.n, [&] {
    if (c->mixed)
      return launch_fluid_f32(c->stream, c->L, c->P, c->mask, c->phi, c->nu32[a], c->h32[a],
                              c->h32[b], c->u32, c->nu32[b], c->tb_a, c->nt_a);
    return launch_fluid_f64(c->stream, c->L, c->P, c->mask, c->phi, c->n[a], c->f[a], c->f[b],
                            c->u, c->n[b], c->tb_a, c->nt_a);
  });
  if (rc) return rc;
  // pass B also moves phi to the extrapolated start of this step's solve
  rc = run(c, KK_IONS, c->L.n, [&] {
    if (c->mixed)
      return launch_ions_f32(c->stream, c->L, c->P, c->mask, c->u32, c->nu32[a], c->lo32[a],
                             c->nu32[b], c->lo32[b], c->src, order, c->phi, keep, c->tb_b,
                             c->nt_b);
    return launch_ions_f64(c->stream, c->L, c->P, c->mask, c->u, c->n[a], c->n[b], c->src,
                           order, c->phi, keep, c->tb_b, c->nt_b);
  });
  return rc;
}

int one_step(lbe_ctx *c, bool record = true) {
  const int a = c->cur, b = 1 - c->cur;
  const int hist = c->extrap_hist;
  // room for this step's charge row before anything moves
  if (record) {
    const int rc = grow_history(c);
    if (rc) return rc;
  }
  int rc = step_passes(c, a, b, hist);
  if (rc) return rc;
  if (c->phi_prev) c->extrap_hist = std::min(hist + 1, 2);
  c->cur = b;
  if (record) {
    c->step++;
    c->charge_dst = c->qhist + c->qlen * std::max(c->ne, 1);
    c->charge_queued = false;
  }
  rc = poisson_solve(c, true);
  c->charge_dst = nullptr;
  if (rc == LBE_ENOCONV || rc == LBE_ENONFINITE) {
    const int rc2 = rewind_step(c, a, hist, record);
    return rc2 ? rc2 : rc;
  }
  if (rc) return rc;
  if (!record) return LBE_OK;
  if (c->charge_queued) {  // already computed behind the solve's last units
    c->qlen++;
    return LBE_OK;
  }
  return record_charge(c);
}

// ---- reverse mode -----------------------------------------------------------

inline size_t pad256(size_t b) { return (b + 255) & ~(size_t)255; }

// Byte layout of a saved state.  A checkpoint holds the populations and
// concentrations in the context's storage (FP64, or the FP32 deviations of
// the mixed form with the low words of the concentration pairs), phi and,
// under LBE_EXTRAPOLATE, phi(t-1).  A recomputed state of one reverse step
// holds rho and m (4 N FP64: the collision sees the populations only through
// them), the concentrations (the high words in the mixed form: the reverse
// step linearises about them) and phi.
struct StateLayout {
  size_t f, n, lo, phi, prev, bytes;
};

StateLayout checkpoint_layout(const lbe_ctx *c) {
  const size_t N = c->L.n, sf = c->mixed ? sizeof(float) : sizeof(double);
  StateLayout l;
  l.f = 0;
  l.n = pad256(NQ * N * sf);
  l.lo = l.n + pad256(c->K * N * sf);
  l.phi = l.lo + (c->mixed ? pad256(c->K * N * sizeof(float)) : 0);
  l.prev = l.phi + pad256(N * sizeof(double));
  l.bytes = l.prev + (c->phi_prev ? pad256(2 * N * sizeof(double)) : 0);
  return l;
}

StateLayout slot_layout(const lbe_ctx *c) {
  const size_t N = c->L.n, sf = c->mixed ? sizeof(float) : sizeof(double);
  StateLayout l;
  l.f = 0;
  l.n = pad256(4 * N * sizeof(double));
  l.lo = l.phi = l.n + pad256(c->K * N * sf);
  l.prev = l.bytes = l.phi + pad256(N * sizeof(double));
  return l;
}

void *cur_pops(lbe_ctx *c) { return c->mixed ? (void *)c->h32[c->cur] : (void *)c->f[c->cur]; }
void *cur_concs(lbe_ctx *c) { return c->mixed ? (void *)c->nu32[c->cur] : (void *)c->n[c->cur]; }

int copy_dd(lbe_ctx *c, void *dst, const void *src, size_t bytes) {
  HIPCHK(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->stream));
  return LBE_OK;
}

int save_state(lbe_ctx *c, char *dst) {
  const StateLayout l = checkpoint_layout(c);
  const size_t N = c->L.n, sf = c->mixed ? sizeof(float) : sizeof(double);
  int rc;
  if ((rc = copy_dd(c, dst + l.f, cur_pops(c), NQ * N * sf)) ||
      (rc = copy_dd(c, dst + l.n, cur_concs(c), c->K * N * sf)) ||
      (rc = copy_dd(c, dst + l.phi, c->phi, N * sizeof(double))))
    return rc;
  if (c->mixed && (rc = copy_dd(c, dst + l.lo, c->lo32[c->cur], c->K * N * sizeof(float))))
    return rc;
  if (c->phi_prev) return copy_dd(c, dst + l.prev, c->phi_prev, 2 * N * sizeof(double));
  return LBE_OK;
}

int load_state(lbe_ctx *c, const char *src) {
  const StateLayout l = checkpoint_layout(c);
  const size_t N = c->L.n, sf = c->mixed ? sizeof(float) : sizeof(double);
  int rc;
  if ((rc = copy_dd(c, cur_pops(c), src + l.f, NQ * N * sf)) ||
      (rc = copy_dd(c, cur_concs(c), src + l.n, c->K * N * sf)) ||
      (rc = copy_dd(c, c->phi, src + l.phi, N * sizeof(double))))
    return rc;
  if (c->mixed && (rc = copy_dd(c, c->lo32[c->cur], src + l.lo, c->K * N * sizeof(float))))
    return rc;
  if (c->phi_prev) return copy_dd(c, c->phi_prev, src + l.prev, 2 * N * sizeof(double));
  return LBE_OK;
}

// the current state as a reverse step needs it
int save_slot(lbe_ctx *c, char *dst) {
  const StateLayout l = slot_layout(c);
  const size_t N = c->L.n, sf = c->mixed ? sizeof(float) : sizeof(double);
  int rc = run(c, KK_ADJ_MOMENTS, c->L.n, [&] {
    double *rhom = (double *)(dst + l.f);
    if (c->mixed)
      return launch_adj_moments<float>(c->stream, c->L, c->P, c->mask, c->h32[c->cur], rhom);
    return launch_adj_moments<double>(c->stream, c->L, c->P, c->mask, c->f[c->cur], rhom);
  });
  if (rc || (rc = copy_dd(c, dst + l.n, cur_concs(c), c->K * N * sf))) return rc;
  return copy_dd(c, dst + l.phi, c->phi, N * sizeof(double));
}

int adjoint_buffers(lbe_ctx *c) {
  const size_t N = c->L.n, K = c->K;
  if (!c->fbar) {
    int rc;
    for (int s = 0; s < 2; ++s) {
      if ((rc = dalloc(c, &c->abar[s], NQ * N))) return rc;
      if ((rc = dalloc(c, &c->nbar[s], K * N))) return rc;
    }
    if ((rc = dalloc(c, &c->lam, N)) || (rc = dalloc(c, &c->lam_sum, N)) ||
        (rc = dalloc(c, &c->gphis, N)) || (rc = dalloc(c, &c->src_keep, N)) ||
        (rc = dalloc(c, &c->adj_u, 3 * N)) || (rc = dalloc(c, &c->qbar_d, std::max(c->ne, 1))) ||
        (rc = dalloc(c, &c->lb_acc, 1)) || (rc = dalloc(c, &c->type_d, N)))
      return rc;
    HIPCHK(c, hipMemcpyAsync(c->type_d, c->type_h.data(), N, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // fbar is allocated last: its presence marks the set complete
    if ((rc = dalloc(c, &c->fbar, 3 * N))) return rc;
  }
  const int slots = (int)std::min<int64_t>(c->tape.every, std::max<int64_t>(c->tape.nsteps, 1));
  if (c->tape.seg_cap < slots) {
    if (c->tape.seg) (void)hipFree(c->tape.seg);
    c->tape.seg = nullptr;
    c->tape.seg_cap = 0;
    int rc = dalloc(c, &c->tape.seg, (size_t)slots * slot_layout(c).bytes);
    if (rc) return rc;
    c->tape.seg_cap = slots;
  }
  return LBE_OK;
}

// Poisson adjoint: L_h lambda = phib with zero wall values; phib arrives as
// the source -phib/6 in c->src, the warm start in c->lam.  Leaves lambda in
// c->phi.  Keeps its own iteration count for the queue of the next adjoint
// solve.
int adjoint_solve(lbe_ctx *c) {
  HIPCHK(c, hipMemcpyAsync(c->phi, c->lam, sizeof(double) * c->L.n, hipMemcpyDeviceToDevice,
                           c->stream));
  std::swap(c->pred_iters, c->adj_pred);
  const int rc = poisson_solve(c, true);
  std::swap(c->pred_iters, c->adj_pred);
  return rc;
}

template <class S>
int adjoint_fold(lbe_ctx *c, const S *n, double *nbar) {
  return run(c, KK_ADJ_FOLD, c->L.n, [&] {
    return launch_adj_fold<S>(c->stream, c->L, c->P, c->mask, c->phi, n, nbar, c->lam_sum, c->lam,
                              c->partial, c->lb_acc);
  });
}

// The reverse sweep of lbe_adjoint; the caller restores the end state.
template <class S>
int adjoint_sweep(lbe_ctx *c, const double *qbar, const double *ubar, double *grad_phi_s,
                  double *grad_lB, double *grad_n, double *grad_f) {
  lbe_ctx::Tape &T = c->tape;
  const size_t N = c->L.n, K = c->K;
  const StateLayout ck = checkpoint_layout(c), sl = slot_layout(c);
  int rc;
  int cur = 0;
  HIPCHK(c, hipMemsetAsync(c->abar[0], 0, sizeof(double) * NQ * N, c->stream));
  HIPCHK(c, hipMemsetAsync(c->abar[1], 0, sizeof(double) * NQ * N, c->stream));
  HIPCHK(c, hipMemsetAsync(c->nbar[0], 0, sizeof(double) * K * N, c->stream));
  HIPCHK(c, hipMemsetAsync(c->nbar[1], 0, sizeof(double) * K * N, c->stream));
  HIPCHK(c, hipMemsetAsync(c->lam, 0, sizeof(double) * N, c->stream));
  HIPCHK(c, hipMemsetAsync(c->lam_sum, 0, sizeof(double) * N, c->stream));
  HIPCHK(c, hipMemsetAsync(c->lb_acc, 0, sizeof(double), c->stream));
  HIPCHK(c, hipMemsetAsync(c->src, 0, sizeof(double) * N, c->stream));
  HIPCHK(c, hipMemsetAsync(c->adj_u, 0, sizeof(double) * 3 * N, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->qbar_d, qbar, sizeof(double) * c->ne, hipMemcpyHostToDevice,
                           c->stream));
  // the momentum term: seed A and Fb, then carry Fb through the link fluxes
  // of the end state (zero concentration adjoint) into nb and the source
  if (ubar[0] != 0.0 || ubar[1] != 0.0 || ubar[2] != 0.0) {
    if ((rc = run(c, KK_ADJ_SEED, c->L.n, [&] {
           return launch_adj_seed_momentum(c->stream, c->L, c->mask, ubar, c->abar[0], c->fbar);
         })))
      return rc;
    if ((rc = run(c, KK_ADJ_IONS, c->L.n, [&] {
           return launch_adj_ions<S>(c->stream, c->L, c->P, c->mask, c->phi,
                                     (const S *)cur_concs(c), c->adj_u, c->fbar, c->nbar[1],
                                     c->nbar[0], c->src);
         })))
      return rc;
  }
  // dQ_e/dl_B = -Q_e / l_B at fixed potential (Eq. 16)
  std::vector<double> qend(c->ne);
  HIPCHK(c, hipMemcpyAsync(qend.data(), c->qhist + (c->qlen - 1) * c->ne,
                           sizeof(double) * c->ne, hipMemcpyDeviceToHost, c->stream));
  const double q_scale = -6.0 / (4.0 * M_PI * c->p.lB);
  if ((rc = run(c, KK_ADJ_SEED, c->L.n, [&] {
         return launch_adj_seed(c->stream, c->L, q_scale, c->mask, c->type_d, c->qbar_d, c->src,
                                c->gphis);
       })))
    return rc;
  HIPCHK(c, hipStreamSynchronize(c->stream));  // qbar and qend
  double lb_explicit = 0.0;
  for (int e = 0; e < c->ne; ++e) lb_explicit -= qbar[e] * qend[e] / c->p.lB;
  // phi(T) depends on n(T): fold its adjoint in
  if ((rc = adjoint_solve(c))) return rc;
  if ((rc = adjoint_fold<S>(c, (const S *)cur_concs(c), c->nbar[cur]))) return rc;
  for (int sg = T.nck - 1; sg >= 0; --sg) {
    const int64_t a = (int64_t)sg * T.every;
    const int64_t b = std::min<int64_t>(a + T.every, T.nsteps);
    if ((rc = load_state(c, T.ck + (size_t)sg * ck.bytes))) return rc;
    c->extrap_hist = T.hist[(size_t)sg];
    for (int64_t t = a; t < b; ++t) {
      if ((rc = save_slot(c, T.seg + (size_t)(t - a) * sl.bytes))) return rc;
      if (t + 1 < b && (rc = one_step(c, false))) return rc;
    }
    for (int64_t t = b - 1; t >= a; --t) {
      const char *slot = T.seg + (size_t)(t - a) * sl.bytes;
      const double *rhom = (const double *)(slot + sl.f);
      const S *ns = (const S *)(slot + sl.n);
      const double *ps = (const double *)(slot + sl.phi);
      const int nxt = 1 - cur;
      if ((rc = run(c, KK_ADJ_FLUID, c->L.n, [&] {
             return launch_adj_fluid<S>(c->stream, c->L, c->P, c->mask, ps, ns, rhom,
                                        c->abar[cur], c->nbar[cur], c->abar[nxt], c->fbar,
                                        c->adj_u);
           })))
        return rc;
      if ((rc = run(c, KK_ADJ_IONS, c->L.n, [&] {
             return launch_adj_ions<S>(c->stream, c->L, c->P, c->mask, ps, ns, c->adj_u, c->fbar,
                                       c->nbar[cur], c->nbar[nxt], c->src);
           })))
        return rc;
      if ((rc = adjoint_solve(c))) return rc;
      if ((rc = adjoint_fold<S>(c, ns, c->nbar[nxt]))) return rc;
      cur = nxt;
    }
  }
  if ((rc = run(c, KK_ADJ_SEED, c->L.n, [&] {
         return launch_adj_phis(c->stream, c->L, c->mask, c->lam_sum, c->gphis);
       })))
    return rc;
  double lb_sweep = 0.0;
  HIPCHK(c, hipMemcpyAsync(&lb_sweep, c->lb_acc, sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
  if (grad_phi_s)
    HIPCHK(c, hipMemcpyAsync(grad_phi_s, c->gphis, sizeof(double) * N, hipMemcpyDeviceToHost,
                             c->stream));
  if (grad_n)
    HIPCHK(c, hipMemcpyAsync(grad_n, c->nbar[cur], sizeof(double) * K * N, hipMemcpyDeviceToHost,
                             c->stream));
  if (grad_f)
    HIPCHK(c, hipMemcpyAsync(grad_f, c->abar[cur], sizeof(double) * NQ * N,
                             hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (grad_lB) *grad_lB = lb_explicit + lb_sweep;
  return LBE_OK;
}

// phi, n, u and f of the current state into caller buffers (host memory for
// kind = hipMemcpyDeviceToHost, device memory for hipMemcpyDeviceToDevice);
// NULL skips one.  Synchronises the stream before returning.
int copy_fields(lbe_ctx *c, double *phi, double *n, double *u, double *f, hipMemcpyKind kind) {
  const long N = c->L.n;
  const int K = c->K;
  int rc;
  if (u || f) {
    // FP64 form: the next step's output buffers are free between steps
    double *fpre = c->mixed ? c->obs : c->f[1 - c->cur];
    double *uo = c->mixed ? c->obs + (size_t)NQ * N : c->u;
    rc = run(c, KK_OBSERVE, c->L.n, [&] {
      if (c->mixed)
        return launch_observe_f32(c->stream, c->L, c->P, c->mask, c->phi, c->nu32[c->cur],
                                  c->h32[c->cur], fpre, uo);
      return launch_observe_f64(c->stream, c->L, c->P, c->mask, c->phi, c->n[c->cur],
                                c->f[c->cur], fpre, uo);
    });
    if (rc) return rc;
    if (f) HIPCHK(c, hipMemcpyAsync(f, fpre, sizeof(double) * NQ * N, kind, c->stream));
    if (u) HIPCHK(c, hipMemcpyAsync(u, uo, sizeof(double) * 3 * N, kind, c->stream));
  }
  if (phi) HIPCHK(c, hipMemcpyAsync(phi, c->phi, sizeof(double) * N, kind, c->stream));
  std::vector<float> nu_h;
  if (n) {
    if (!c->mixed) {
      HIPCHK(c, hipMemcpyAsync(n, c->n[c->cur], sizeof(double) * K * N, kind, c->stream));
    } else if (kind == hipMemcpyDeviceToDevice) {
      rc = run(c, KK_EXPAND_N, c->L.n, [&] {
        return launch_expand_n_f32(c->stream, c->L, c->P, c->mask, c->nu32[c->cur],
                                   c->lo32[c->cur], n);
      });
      if (rc) return rc;
    } else {
      nu_h.resize((size_t)2 * K * N);
      HIPCHK(c, hipMemcpyAsync(nu_h.data(), c->nu32[c->cur], sizeof(float) * K * N,
                               hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipMemcpyAsync(nu_h.data() + (size_t)K * N, c->lo32[c->cur],
                               sizeof(float) * K * N, hipMemcpyDeviceToHost, c->stream));
    }
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (!nu_h.empty())
    for (int k = 0; k < K; ++k)
      for (long r = 0; r < N; ++r) {
        const size_t i = (size_t)k * N + r;
        n[i] = c->type_h[r] ? 0.0
                            : c->nref_h[(size_t)c->sys_h[r] * 4 + k] +
                                  ((double)nu_h[i] + (double)nu_h[(size_t)K * N + i]);
      }
  return LBE_OK;
}

// true when p is device memory of device dev (-1: the current device)
bool on_device(const void *p, int dev = -1) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  if (dev < 0) (void)hipGetDevice(&dev);
  return (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged) && a.device == dev;
}

void free_ctx(lbe_ctx *c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  void *ptrs[] = {c->mask, c->phi, c->phi_prev, c->phi_keep, c->src, c->u, c->n[0], c->n[1], c->f[0], c->f[1],
                  c->h32[0], c->h32[1], c->nu32[0], c->nu32[1], c->lo32[0], c->lo32[1],
                  c->u32, c->obs,
                  c->partial, c->dout, c->ctl, c->iface, c->blk_elec, c->blk_begin,
                  c->blk_end, c->qcur, c->qhist, c->solid_idx, c->solid_val,
                  c->nref_d_tab, c->qref_tab, c->nref_f_tab, c->kr, c->kp, c->kq, c->kaz, c->kc,
                  c->tape.ck, c->tape.seg, c->abar[0], c->abar[1], c->nbar[0], c->nbar[1],
                  c->fbar, c->adj_u, c->lam, c->lam_sum, c->gphis, c->src_keep, c->qbar_d,
                  c->lb_acc, c->type_d};
  for (void *q : ptrs)
    if (q) (void)hipFree(q);
  for (auto &L : c->mg) {
    if (L.own_mask && L.mask) (void)hipFree(L.mask);
    if (L.e) (void)hipFree(L.e);
    if (L.e2) (void)hipFree(L.e2);
    if (L.r) (void)hipFree(L.r);
  }
  if (c->unit_exec) (void)hipGraphExecDestroy(c->unit_exec);
  if (c->chunk_exec) (void)hipGraphExecDestroy(c->chunk_exec);
  if (c->chunk_q) (void)hipFree(c->chunk_q);
  if (c->chunk_st) (void)hipFree(c->chunk_st);
  if (c->mg_ainv) (void)hipFree(c->mg_ainv);
  if (c->mg_fcell) (void)hipFree(c->mg_fcell);
  if (c->mg_groups) (void)hipFree(c->mg_groups);
  if (c->hpin) (void)hipHostFree(c->hpin);
  if (c->ctl_h) (void)hipHostFree(c->ctl_h);
  if (c->ctl_pub) (void)hipHostFree(c->ctl_pub);
  for (int k = 0; k < KK_COUNT; ++k)
    for (auto &pr : c->pending[k]) {
      (void)hipEventDestroy(pr.a);
      (void)hipEventDestroy(pr.b);
    }
  for (auto e : c->pool) (void)hipEventDestroy(e);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

}  // namespace

// ---- public API -------------------------------------------------------------

extern "C" {

const char *lbe_strerror(int code) {
  switch (code) {
    case LBE_OK: return "ok";
    case LBE_EINVAL: return "invalid argument";
    case LBE_EGEOM: return "invalid geometry";
    case LBE_ENOMEM: return "out of memory";
    case LBE_EDEVICE: return "device error";
    case LBE_ENOCONV: return "Poisson solve did not converge";
    case LBE_ENONFINITE: return "non-finite value";
    default: return "unknown error";
  }
}

const char *lbe_last_error(const lbe_ctx *c) { return c ? c->err.c_str() : g_init_error.c_str(); }

#ifndef LBE_BUILD_ID
#define LBE_BUILD_ID "unknown"
#endif
const char *lbe_build_id(void) { return LBE_BUILD_ID; }

void lbe_velocities(int32_t *c, double *w) {
  for (int i = 0; i < NQ; ++i) {
    if (c) {
      c[3 * i] = CX[i];
      c[3 * i + 1] = CY[i];
      c[3 * i + 2] = CZ[i];
    }
    if (w) w[i] = WQ[i];
  }
}

int32_t lbe_num_kernel_kinds(void) { return KK_COUNT; }

int lbe_launch_shape(const lbe_ctx *c, int32_t *block_a, int32_t *block_b, int32_t *nontemporal) {
  if (!c) return fail(nullptr, LBE_EINVAL, "context is NULL");
  if (block_a) *block_a = c->tb_a;
  if (block_b) *block_b = c->tb_b;
  if (nontemporal) *nontemporal = (c->nt_a ? 1 : 0) | (c->nt_b ? 2 : 0);
  return LBE_OK;
}
const char *lbe_kernel_name(int32_t kind) {
  return (kind >= 0 && kind < KK_COUNT) ? kKernelNames[kind] : "";
}

}  // extern "C"

namespace {

// lbe_init and lbe_init_batch: system == nullptr means one system (nsys = 1).
// Launch shape of the two step passes, picked by timing: each candidate
// block size runs pass A, then pass B, on scratch outputs (the next step's
// buffers; for pass B also a scratch source and a scratch copy of phi), best
// of three launches after one to warm up.  Every site is computed on its own,
// so the results are the same for any choice; only the time differs.
int autotune_passes(lbe_ctx *c) {
  static const int cand_all[4] = {128, 256, 512, TB_TILED};
  const int a = c->cur, b = 1 - c->cur;
  const long N = c->L.n;
  // scratch for pass B's source and kept potential: free between steps
  double *src_s = c->mixed ? c->obs : c->f[b];
  double *keep_s = src_s + N;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(c, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(c, LBE_EDEVICE, "event create failed");
  }
  // The LDS-staged forms of the passes where their tiles fit the lattice.
  // Pass B's tiles are a timed candidate (in the FP64 form for one or two
  // species, whose values fill 54 KB of LDS).  The mixed pass A's plane rings
  // pay only where the populations stream from HBM (they overflow the
  // 256 MB last-level cache): on the 192^3 porous electrode 301 us against
  // 317 us for the best block size, in a running state, while the trial
  // launches from the initial state tell the two apart by less than their
  // noise; on the cache-resident 160 x 160 x 64 and 64 x 64 x 130 lattices
  // 97 and 43 us against 81 and 27 us.  So pass A takes them there
  // untimed, and only there.  (The FP64 pass A, bound by its arithmetic,
  // took 648 us on the rings against 624 us: it has none.)  LBE_PASS_TILE=0 leaves both out, =1 takes
  // both untimed where they fit (LBE_PASS_TILE_A, LBE_PASS_TILE_B for one
  // pass).
  const int both = env_flag("LBE_PASS_TILE", -1);
  const bool big = (size_t)NQ * c->L.n * (c->mixed ? sizeof(float) : sizeof(double)) >
                   ((size_t)256 << 20);
  const int tile_env[2] = {env_flag("LBE_PASS_TILE_A", both >= 0 ? both : (big ? 1 : 0)),
                           env_flag("LBE_PASS_TILE_B", both)};
  const bool tile_ok[2] = {c->mixed && rings_fit(c->L) && tile_env[0] != 0,
                           (c->mixed || c->P.K <= 2) && tiles_fit(c->L) && tile_env[1] != 0};
  int rc = LBE_OK;
  for (int pass = 0; pass < 2 && rc == LBE_OK; ++pass) {
    float best = 1e30f;
    int pick = 256;
    for (int tb : cand_all) {
      if (tb == TB_TILED && !tile_ok[pass]) continue;
      if (tile_ok[pass] && tile_env[pass] == 1 && tb != TB_TILED) continue;
      float t_min = 1e30f;
      for (int rep = 0; rep < 4 && rc == LBE_OK; ++rep) {
        hipError_t e = hipEventRecord(e0, c->stream);
        if (e == hipSuccess) {
          if (pass == 0)
            e = c->mixed ? launch_fluid_f32(c->stream, c->L, c->P, c->mask, c->phi, c->nu32[a],
                                            c->h32[a], c->h32[b], c->u32, c->nu32[b], tb, c->nt_a)
                         : launch_fluid_f64(c->stream, c->L, c->P, c->mask, c->phi, c->n[a],
                                            c->f[a], c->f[b], c->u, c->n[b], tb, c->nt_a);
          else
            e = c->mixed ? launch_ions_f32(c->stream, c->L, c->P, c->mask, c->u32, c->nu32[a],
                                           c->lo32[a], c->nu32[b], c->lo32[b], src_s, -1,
                                           c->phi, keep_s, tb, c->nt_b)
                         : launch_ions_f64(c->stream, c->L, c->P, c->mask, c->u, c->n[a],
                                           c->n[b], src_s, -1, c->phi, keep_s, tb, c->nt_b);
        }
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
          rc = hip_fail(c, e, "pass timing");
          break;
        }
        if (rep > 0) t_min = std::min(t_min, ms);
      }
      if (t_min < best) {
        best = t_min;
        pick = tb;
      }
    }
    (pass == 0 ? c->tb_a : c->tb_b) = pick;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

int init_impl(const lbe_params *params, const uint8_t *type, const double *phi_s,
              const double *n_init, const double *n_ref, const double *f_init,
              const uint16_t *system, int nsys, lbe_ctx **out) {
  g_init_error.clear();
  if (!out) return fail(nullptr, LBE_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(params);
  if (rc) return rc;
  if (!type || !phi_s) return fail(nullptr, LBE_EINVAL, "type and phi_s are required");
  const lbe_params &p = *params;
  const long N = (long)p.nx * p.ny * p.nz;
  const int K = p.nspecies;
  int ne = 0;
  for (long r = 0; r < N; ++r) ne = std::max(ne, (int)type[r]);
  if (ne > LBE_MAX_ELECTRODES) return fail(nullptr, LBE_EINVAL, "too many electrodes");
  if (nsys < 1 || nsys > LBE_MAX_SYSTEMS) return fail(nullptr, LBE_EINVAL, "bad system count");
  std::vector<uint16_t> sys_h(N, 0);
  if (system)
    for (long r = 0; r < N; ++r) {
      if (type[r]) continue;
      if (system[r] >= nsys) return fail(nullptr, LBE_EINVAL, "system index out of range");
      sys_h[r] = system[r];
    }
  for (long r = 0; r < N; ++r)
    if (type[r] && !isfinite(phi_s[r]))
      return fail(nullptr, LBE_EINVAL, "non-finite electrode potential");
  if (!n_init && !n_ref) return fail(nullptr, LBE_EINVAL, "n_init or n_ref is required");
  std::vector<double> n0((size_t)K * N, 0.0);
  for (int k = 0; k < K; ++k)
    for (long r = 0; r < N; ++r) {
      if (type[r]) continue;
      const double v = n_init ? n_init[(size_t)k * N + r] : n_ref[(size_t)sys_h[r] * K + k];
      if (!isfinite(v)) return fail(nullptr, LBE_EINVAL, "non-finite initial concentration");
      n0[(size_t)k * N + r] = v;
    }
  // populations in pull form: stored_i(r - c_i) = f_i(r), or the node's own
  // opposite slot when r - c_i is solid
  std::vector<double> fs((size_t)NQ * N, 0.0);
  for (long r = 0; r < N; ++r) {
    if (type[r]) continue;
    const int z = (int)(r / ((long)p.nx * p.ny));
    const int rem = (int)(r - (long)z * p.nx * p.ny);
    const int y = rem / p.nx, x = rem - y * p.nx;
    for (int i = 0; i < NQ; ++i) {
      const double v = f_init ? f_init[(size_t)i * N + r] : WQ[i] * p.rho0;
      if (!isfinite(v)) return fail(nullptr, LBE_EINVAL, "non-finite initial population");
      const long rs = wrap(x - CX[i], p.nx) + (long)p.nx * (wrap(y - CY[i], p.ny) + (long)p.ny * wrap(z - CZ[i], p.nz));
      if (i == 0) fs[r] = v;
      else if (type[rs]) fs[(size_t)OPP[i] * N + r] = v;
      else fs[(size_t)i * N + rs] = v;
    }
  }
  HostGeometry g;
  rc = build_geometry(&p, type, sys_h.data(), ne, g);
  if (rc) return rc;

  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
    return fail(nullptr, LBE_EDEVICE, "no HIP device");
  lbe_ctx *c = new lbe_ctx();
  c->p = p;
  c->K = K;
  c->ne = ne;
  (void)hipGetDevice(&c->device);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) != hipSuccess ||
      strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    std::string arch = prop.gcnArchName;
    free_ctx(c);
    return fail(nullptr, LBE_EDEVICE, "library is built for gfx950, device is " + arch);
  }
  {
    // stencil kernels give each die a contiguous run of blocks (same results)
    const char *nx = getenv("LBE_NO_XCD_MAP");
    c->L = make_lattice(p.nx, p.ny, p.nz, g.selfm,
                        (p.flags & LBE_NAIVE_DIRICHLET) ? 1.0 : 2.0,
                        (nx && *nx && *nx != '0') ? 0 : 1);
  }
  c->P.K = K;
  for (int k = 0; k < K; ++k) {
    c->P.z[k] = p.z[k];
    c->P.dk[k] = p.D[k] / A0;
  }
  for (int i = 0; i < NQ; ++i)
    c->P.Ec[i] = p.Eapp[0] * CX[i] + p.Eapp[1] * CY[i] + p.Eapp[2] * CZ[i];
  c->P.tau = p.tau;
  c->P.src_scale = 4.0 * M_PI * p.lB / 6.0;
  c->P.omega = p.omega;
  c->mixed = p.precision == LBE_FP32_MIXED;
  {
    const char *ng = getenv("LBE_NO_GRAPHS");
    c->use_graphs = !(ng && *ng && *ng != '0');
    const char *nt = getenv("LBE_NO_TILES");  // the eight-lane restriction only (same results)
    c->tiles = !(nt && *nt && *nt != '0');
    // the stencil kernels gathering from global memory (same results, the
    // Krylov sums aside), or their plane rings at a given run length on every
    // level that fits them
    const char *nr = getenv("LBE_NO_RINGS");
    const char *zr = getenv("LBE_RING_ZRUN");
    c->rings = (nr && *nr && *nr != '0') ? RING_OFF : (zr && atoi(zr) > 0 ? atoi(zr) : RING_AUTO);
    // the coarse levels' first sweep as a separate launch (same results)
    const char *ns = getenv("LBE_NO_COARSE_START");
    c->coarse_start = !(ns && *ns && *ns != '0');
    c->mg_jacobi = p.mg_smoother == LBE_MG_JACOBI ? 1.0 : 0.0;
    const bool same = p.mg_nu1_coarse == 0 && p.mg_nu2_coarse == 0;
    c->mg_nu1c = same ? p.mg_nu1 : p.mg_nu1_coarse;
    c->mg_nu2c = same ? p.mg_nu2 : p.mg_nu2_coarse;
  }
  c->type_h.assign(type, type + N);
  c->sys_h = sys_h;
  // references of the mixed form per system: n_ref, else the system's fluid
  // mean of n_init
  {
    std::vector<double> sum((size_t)nsys * 4, 0.0);
    std::vector<long> cnt(nsys, 0);
    for (long r = 0; r < N; ++r) {
      if (type[r]) continue;
      cnt[sys_h[r]]++;
      for (int k = 0; k < K; ++k) sum[(size_t)sys_h[r] * 4 + k] += n0[(size_t)k * N + r];
    }
    c->nref_h.assign((size_t)nsys * 4, 0.0);
    for (int sy = 0; sy < nsys; ++sy)
      for (int k = 0; k < K; ++k) {
        double ref = n_ref ? n_ref[(size_t)sy * K + k]
                           : (cnt[sy] ? sum[(size_t)sy * 4 + k] / (double)cnt[sy] : 0.0);
        if (!isfinite(ref)) {
          free_ctx(c);
          return fail(nullptr, LBE_EINVAL, "non-finite reference concentration");
        }
        c->nref_h[(size_t)sy * 4 + k] = ref;
      }
    for (int k = 0; k < K; ++k) c->P.dk_f[k] = (float)c->P.dk[k];
    c->P.unit_z = 1;
    for (int k = 0; k < K; ++k)
      if (p.z[k] != 1 && p.z[k] != -1) c->P.unit_z = 0;
    c->P.rho0_d = p.rho0;
    c->P.rho0_f = (float)p.rho0;
    c->P.itau_f = (float)(1.0 / p.tau);
  }

#define TRY(x)          \
  do {                  \
    rc = (x);           \
    if (rc) goto fail_; \
  } while (0)
  if (p.stream) {
    c->stream = (hipStream_t)p.stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      rc = fail(c, LBE_EDEVICE, "stream creation failed");
      goto fail_;
    }
    c->own_stream = true;
  }
  {
    const int nres = residual_blocks(c->L);
    const int ntot = totals_blocks(c->L) * (2 + K);
    // the Krylov iteration's four sums take 4 partials per block
    const int npart = std::max({nres, ntot, 4 * totals_blocks(c->L), (int)g.blk_elec.size(), 1});
    TRY(dalloc(c, &c->mask, N));
    TRY(dalloc(c, &c->phi, N));
    TRY(dalloc(c, &c->src, N));
    {
      std::vector<float> rf(c->nref_h.begin(), c->nref_h.end());
      std::vector<double> qr(nsys, 0.0);
      for (int sy = 0; sy < nsys; ++sy)
        for (int k = 0; k < K; ++k) qr[sy] += p.z[k] * c->nref_h[(size_t)sy * 4 + k];
      TRY(dalloc(c, &c->nref_d_tab, c->nref_h.size()));
      TRY(dalloc(c, &c->nref_f_tab, rf.size()));
      TRY(dalloc(c, &c->qref_tab, qr.size()));
      if (hipMemcpy(c->nref_d_tab, c->nref_h.data(), sizeof(double) * c->nref_h.size(),
                    hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(c->nref_f_tab, rf.data(), sizeof(float) * rf.size(), hipMemcpyHostToDevice) !=
              hipSuccess ||
          hipMemcpy(c->qref_tab, qr.data(), sizeof(double) * qr.size(), hipMemcpyHostToDevice) !=
              hipSuccess) {
        rc = fail(c, LBE_EDEVICE, "copy of the reference tables failed");
        goto fail_;
      }
      c->P.nref_d = c->nref_d_tab;
      c->P.nref_f = c->nref_f_tab;
      c->P.qref = c->qref_tab;
      c->qref_h = qr;
    }
    if (c->mixed) {
      TRY(dalloc(c, &c->u32, 3 * N));
      TRY(dalloc(c, &c->obs, (size_t)(NQ + 3) * N));
      for (int s = 0; s < 2; ++s) {
        TRY(dalloc(c, &c->nu32[s], (size_t)K * N));
        TRY(dalloc(c, &c->lo32[s], (size_t)K * N));
        TRY(dalloc(c, &c->h32[s], (size_t)NQ * N));
      }
    } else {
      TRY(dalloc(c, &c->u, 3 * N));
      for (int s = 0; s < 2; ++s) {
        TRY(dalloc(c, &c->n[s], (size_t)K * N));
        TRY(dalloc(c, &c->f[s], (size_t)NQ * N));
      }
    }
    TRY(dalloc(c, &c->partial, npart));
    TRY(dalloc(c, &c->dout, 16));
    TRY(dalloc(c, &c->ctl, 1));
    if (hipHostMalloc((void **)&c->ctl_h, sizeof(SolveCtl)) != hipSuccess) {
      rc = fail(c, LBE_ENOMEM, "pinned host buffer");
      goto fail_;
    }
    // the published copy: coherent, device-mapped host memory (optional)
    if (hipHostMalloc((void **)&c->ctl_pub, sizeof(SolveCtl),
                      hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess ||
        hipHostGetDevicePointer((void **)&c->ctl_pub_d, c->ctl_pub, 0) != hipSuccess) {
      (void)hipGetLastError();
      if (c->ctl_pub) (void)hipHostFree(c->ctl_pub);
      c->ctl_pub = nullptr;
      c->ctl_pub_d = nullptr;
    } else {
      memset((void *)c->ctl_pub, 0, sizeof(SolveCtl));  // the stamp of no solve
    }
    TRY(dalloc(c, &c->iface, g.iface.size()));
    TRY(dalloc(c, &c->blk_elec, g.blk_elec.size()));
    TRY(dalloc(c, &c->blk_begin, g.blk_begin.size()));
    TRY(dalloc(c, &c->blk_end, g.blk_end.size()));
    TRY(dalloc(c, &c->qcur, std::max(ne, 1)));
    if (hipHostMalloc((void **)&c->hpin, 64 * sizeof(double)) != hipSuccess) {
      rc = fail(c, LBE_ENOMEM, "pinned host buffer");
      goto fail_;
    }
    c->nblk_charge = (int)g.blk_elec.size();

    std::vector<double> phi0(N, 0.0), src0(N, 0.0);
    std::vector<float> nu0, lo0, h0;
    if (c->mixed) {
      nu0.assign((size_t)K * N, 0.f);
      lo0.assign((size_t)K * N, 0.f);
      h0.assign((size_t)NQ * N, 0.f);
      // the pair: hi the deviation rounded to FP32, lo what that rounding left
      for (int k = 0; k < K; ++k)
        for (long r = 0; r < N; ++r)
          if (!type[r]) {
            const size_t i = (size_t)k * N + r;
            const double d = n0[i] - c->nref_h[(size_t)sys_h[r] * 4 + k];
            nu0[i] = (float)d;
            lo0[i] = (float)(d - (double)nu0[i]);
          }
      for (int i = 0; i < NQ; ++i)
        for (long r = 0; r < N; ++r)
          if (!type[r]) h0[(size_t)i * N + r] = (float)(fs[(size_t)i * N + r] - WQ[i] * p.rho0);
    }
    for (long r = 0; r < N; ++r) {
      if (type[r]) {
        phi0[r] = phi_s[r];
        continue;
      }
      double q = 0.0;
      if (c->mixed) {
        q = c->qref_h[sys_h[r]];
        for (int k = 0; k < K; ++k)
          q += p.z[k] * ((double)nu0[(size_t)k * N + r] + (double)lo0[(size_t)k * N + r]);
      } else {
        for (int k = 0; k < K; ++k) q += p.z[k] * n0[(size_t)k * N + r];
      }
      src0[r] = c->P.src_scale * q;
    }
    auto up = [&](void *d, const void *h, size_t bytes) -> int {
      if (!bytes) return LBE_OK;
      HIPCHK(c, hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, c->stream));
      return LBE_OK;
    };
    TRY(up(c->mask, g.mask.data(), sizeof(uint32_t) * N));
    TRY(up(c->phi, phi0.data(), sizeof(double) * N));
    TRY(up(c->src, src0.data(), sizeof(double) * N));
    for (int s = 0; s < 2; ++s) {
      if (c->mixed) {
        TRY(up(c->nu32[s], nu0.data(), sizeof(float) * K * N));
        TRY(up(c->lo32[s], lo0.data(), sizeof(float) * K * N));
        TRY(up(c->h32[s], h0.data(), sizeof(float) * NQ * N));
      } else {
        TRY(up(c->n[s], n0.data(), sizeof(double) * K * N));
        TRY(up(c->f[s], fs.data(), sizeof(double) * NQ * N));
      }
    }
    TRY(up(c->iface, g.iface.data(), sizeof(int) * g.iface.size()));
    TRY(up(c->blk_elec, g.blk_elec.data(), sizeof(int) * g.blk_elec.size()));
    TRY(up(c->blk_begin, g.blk_begin.data(), sizeof(int) * g.blk_begin.size()));
    TRY(up(c->blk_end, g.blk_end.data(), sizeof(int) * g.blk_end.size()));
    if ((c->u && hipMemsetAsync(c->u, 0, sizeof(double) * 3 * N, c->stream) != hipSuccess) ||
        (c->u32 && hipMemsetAsync(c->u32, 0, sizeof(float) * 3 * N, c->stream) != hipSuccess)) {
      rc = fail(c, LBE_EDEVICE, "memset failed");
      goto fail_;
    }
    // synchronous: the host vectors go out of scope
    if (hipStreamSynchronize(c->stream) != hipSuccess) {
      rc = fail(c, LBE_EDEVICE, "stream synchronize failed");
      goto fail_;
    }
  }
  if (p.poisson == LBE_MG || c->mixed) TRY(build_multigrid(c, type, p.poisson != LBE_MG));
  if (p.poisson == LBE_MG && (p.flags & LBE_KRYLOV)) {
    TRY(dalloc(c, &c->kr, N));
    TRY(dalloc(c, &c->kp, N));
    TRY(dalloc(c, &c->kq, N));
    TRY(dalloc(c, &c->kaz, N));
    TRY(dalloc(c, &c->kc, 1));
    if (hipMemsetAsync(c->kp, 0, sizeof(double) * N, c->stream) != hipSuccess ||
        hipMemsetAsync(c->kq, 0, sizeof(double) * N, c->stream) != hipSuccess ||
        hipMemsetAsync(c->kaz, 0, sizeof(double) * N, c->stream) != hipSuccess ||
        hipMemsetAsync(c->kc, 0, sizeof(KrylovCtl), c->stream) != hipSuccess) {
      rc = fail(c, LBE_EDEVICE, "memset failed");
      goto fail_;
    }
  }
  TRY(poisson_solve(c, false));
  TRY(record_charge(c));
  {
    // Non-temporal streams in the step passes when the populations alone
    // overflow the 256 MB last-level cache (on the cache-resident 64x64x130
    // slab they cost 7%).  LBE_NT=0|1 sets both passes, LBE_NT_A, LBE_NT_B
    // one each.
    {
      const bool big = (size_t)NQ * N * (c->mixed ? sizeof(float) : sizeof(double)) >
                       ((size_t)256 << 20);
      const int both = env_flag("LBE_NT", -1);
      c->nt_a = env_flag("LBE_NT_A", both >= 0 ? both : (big ? 1 : 0)) != 0;
      c->nt_b = env_flag("LBE_NT_B", both >= 0 ? both : (big ? 1 : 0)) != 0;
    }
    // LBE_PASS_BLOCK=128|256|512 fixes the passes' block size; LBE_NO_AUTOTUNE
    // keeps 256; otherwise the context times the candidates
    const char *pb = getenv("LBE_PASS_BLOCK");
    const int fixed = pb ? atoi(pb) : 0;
    const char *na = getenv("LBE_NO_AUTOTUNE");
    if (fixed == 128 || fixed == 256 || fixed == 512)
      c->tb_a = c->tb_b = fixed;
    else if (!(na && *na && *na != '0'))
      TRY(autotune_passes(c));
  }
  if (p.flags & LBE_EXTRAPOLATE) {
    TRY(dalloc(c, &c->phi_prev, 2 * N));
    c->extrap_hist = 0;  // the first step starts from phi(0) itself
    if (hipMemsetAsync(c->phi_prev, 0, sizeof(double) * 2 * N, c->stream) != hipSuccess) {
      rc = fail(c, LBE_EDEVICE, "memset failed");
      goto fail_;
    }
  } else {
    TRY(dalloc(c, &c->phi_keep, N));
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess) {
    rc = fail(c, LBE_EDEVICE, "stream synchronize failed");
    goto fail_;
  }
#undef TRY
  *out = c;
  return LBE_OK;
fail_:
  g_init_error = c->err;
  free_ctx(c);
  return rc;
}

}  // namespace

// Capture CHUNK_STEPS whole steps from the current buffers, each with `units`
// solver units, as one graph.  Nothing runs: the host-side state the
// queueing moves (buffer parity, extrapolation history) is put back, and
// since CHUNK_STEPS is even and the history is full, a replay ends where it
// began.
int capture_chunk(lbe_ctx *c, int units) {
  if (c->chunk_exec) {
    (void)hipGraphExecDestroy(c->chunk_exec);
    c->chunk_exec = nullptr;
  }
  const int cur0 = c->cur, hist0 = c->extrap_hist, ne = std::max(c->ne, 1);
  HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  int rc = LBE_OK;
  c->queue_units = units;
  for (int s = 0; s < CHUNK_STEPS && !rc; ++s) {
    const int a = c->cur, b = 1 - a;
    if ((rc = step_passes(c, a, b, c->extrap_hist))) break;
    if (c->phi_prev) c->extrap_hist = std::min(c->extrap_hist + 1, 2);
    c->cur = b;
    // no charge kernel when no electrode touches the fluid (rows filled after)
    c->charge_dst = c->nblk_charge > 0 ? c->chunk_q + (size_t)s * ne : nullptr;
    rc = poisson_solve(c, false);
  }
  c->queue_units = 0;
  c->charge_dst = nullptr;
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(c->stream, &g);
  c->cur = cur0;
  c->extrap_hist = hist0;
  if (rc || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return rc ? rc : hip_fail(c, e, "chunk graph capture");
  }
  const hipError_t e2 = hipGraphInstantiate(&c->chunk_exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e2 != hipSuccess) {
    c->chunk_exec = nullptr;
    return hip_fail(c, e2, "chunk graph instantiate");
  }
  c->chunk_units = units;
  c->chunk_cur = cur0;
  c->chunk_tol = c->p.tol;
  return LBE_OK;
}

extern "C" {

int lbe_init(const lbe_params *params, const uint8_t *type, const double *phi_s,
             const double *n_init, const double *n_ref, const double *f_init, lbe_ctx **out) {
  return init_impl(params, type, phi_s, n_init, n_ref, f_init, nullptr, 1, out);
}

int lbe_init_batch(const lbe_params *params, const uint8_t *type, const double *phi_s,
                   const double *n_init, const double *n_ref, const uint16_t *system,
                   int32_t nsys, lbe_ctx **out) {
  if (!system) {
    g_init_error.clear();
    if (out) *out = nullptr;
    return fail(nullptr, LBE_EINVAL, "system is NULL");
  }
  return init_impl(params, type, phi_s, n_init, n_ref, nullptr, system, nsys, out);
}

int lbe_init_device(const lbe_params *params, const uint8_t *type, const double *phi_s,
                    const double *n_init, const double *n_ref, const double *f_init,
                    lbe_ctx **out) {
  g_init_error.clear();
  if (out) *out = nullptr;
  int rc = validate(params);
  if (rc) return rc;
  if (!type || !phi_s) return fail(nullptr, LBE_EINVAL, "type and phi_s are required");
  if (!n_init && !n_ref) return fail(nullptr, LBE_EINVAL, "n_init or n_ref is required");
  const size_t N = (size_t)params->nx * params->ny * params->nz;
  const size_t K = (size_t)params->nspecies;
  struct Arg {
    const void *src;
    size_t bytes;
  } args[] = {{type, N}, {phi_s, N * sizeof(double)}, {n_init, K * N * sizeof(double)},
              {n_ref, K * sizeof(double)}, {f_init, NQ * N * sizeof(double)}};
  for (const Arg &a : args)
    if (a.src && !on_device(a.src))
      return fail(nullptr, LBE_EINVAL, "an input is not device memory of the current device");
  // the geometry analysis runs on the host: copy the borrowed arrays there
  std::vector<uint8_t> t(N);
  std::vector<double> ps(N), ni(n_init ? K * N : 0), nr(n_ref ? K : 0), fi(f_init ? NQ * N : 0);
  void *dst[] = {t.data(), ps.data(), ni.data(), nr.data(), fi.data()};
  hipStream_t s = (hipStream_t)params->stream;
  for (int i = 0; i < 5; ++i)
    if (args[i].src && hipMemcpyAsync(dst[i], args[i].src, args[i].bytes, hipMemcpyDeviceToHost,
                                      s) != hipSuccess)
      return fail(nullptr, LBE_EDEVICE, "copy of an input failed");
  if (hipStreamSynchronize(s) != hipSuccess)
    return fail(nullptr, LBE_EDEVICE, "stream synchronize failed");
  return init_impl(params, t.data(), ps.data(), n_init ? ni.data() : nullptr,
                   n_ref ? nr.data() : nullptr, f_init ? fi.data() : nullptr, nullptr, 1, out);
}

int lbe_set_solver(lbe_ctx *c, double tol, int32_t max_iter) {
  if (!c) return fail(c, LBE_EINVAL, "context is NULL");
  if (!std::isfinite(tol) || max_iter < 0) return fail(c, LBE_EINVAL, "bad tol or max_iter");
  c->p.tol = tol;
  c->p.max_iter = max_iter;
  return LBE_OK;
}

int lbe_fields_device(lbe_ctx *c, double *phi, double *n, double *u, double *f) {
  if (!c) return fail(c, LBE_EINVAL, "context is NULL");
  for (const void *q : {(const void *)phi, (const void *)n, (const void *)u, (const void *)f})
    if (q && !on_device(q, c->device)) return fail(c, LBE_EINVAL, "an output is not device memory of the context's device");
  return copy_fields(c, phi, n, u, f, hipMemcpyDeviceToDevice);
}

int lbe_step(lbe_ctx *c, int64_t nsteps) {
  if (!c || nsteps < 0) return fail(c, LBE_EINVAL, "bad context or step count");
  for (int64_t t = 0; t < nsteps; ++t) {
    int rc = one_step(c);
    if (rc) return rc;
  }
  return LBE_OK;
}

int lbe_step_chunk(lbe_ctx *c, int64_t nsteps, int32_t units) {
  if (!c || nsteps < 0 || units < 1)
    return fail(c, LBE_EINVAL, "bad context, step count or unit count");
  const lbe_params &p = c->p;
  const int per_check = p.poisson == LBE_MG ? 1 : p.check_every;
  if (!(p.tol > 0.0)) return fail(c, LBE_EINVAL, "graph-replayed steps need a tolerance > 0");
  if ((int64_t)units * per_check > (int64_t)p.max_iter)
    return fail(c, LBE_EINVAL, "units x iterations per unit exceed max_iter");
  int64_t t = 0;
  int rc;
  // the steps after init or a change of the electrode potentials start from
  // a lower extrapolation order: taken one by one
  for (; t < nsteps && c->phi_prev && c->extrap_hist < 2; ++t)
    if ((rc = one_step(c))) return rc;
  const int64_t reps = (c->prof || !c->use_graphs) ? 0 : (nsteps - t) / CHUNK_STEPS;
  if (reps > 0) {
    const int ne = std::max(c->ne, 1);
    if ((rc = grow_history(c, c->qlen + reps * CHUNK_STEPS))) return rc;
    if (!c->chunk_q && (rc = dalloc(c, &c->chunk_q, (size_t)CHUNK_STEPS * ne))) return rc;
    if (!c->chunk_st && (rc = dalloc(c, &c->chunk_st, 1))) return rc;
    if (!c->chunk_exec || c->chunk_units != units || c->chunk_cur != c->cur ||
        c->chunk_tol != p.tol)
      if ((rc = capture_chunk(c, units))) return rc;
    HIPCHK(c, hipMemsetAsync(c->chunk_st, 0, sizeof(ChunkStatus), c->stream));
    const size_t rows = (size_t)CHUNK_STEPS * ne;
    for (int64_t r = 0; r < reps; ++r) {
      HIPCHK(c, hipGraphLaunch(c->chunk_exec, c->stream));
      double *dst = c->qhist + (size_t)c->qlen * ne;
      if (c->nblk_charge > 0)
        HIPCHK(c, hipMemcpyAsync(dst, c->chunk_q, sizeof(double) * rows,
                                 hipMemcpyDeviceToDevice, c->stream));
      else
        HIPCHK(c, hipMemsetAsync(dst, 0, sizeof(double) * rows, c->stream));
      c->qlen += CHUNK_STEPS;
      c->step += CHUNK_STEPS;
    }
    ChunkStatus st{};
    HIPCHK(c, hipMemcpyAsync(&st, c->chunk_st, sizeof st, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->ctl_h, c->ctl, sizeof(SolveCtl), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->last_iters = c->ctl_h->done ? c->ctl_h->iters : c->ctl_h->count;
    c->last_resid = c->ctl_h->resid;
    c->total_iters += st.iters;
    if (st.nonfinite) return fail(c, LBE_ENONFINITE, "non-finite Poisson residual in a replayed step");
    if (st.unconverged) {
      char buf[200];
      snprintf(buf, sizeof buf,
               "Poisson not converged in %d of %lld replayed steps with %d units each "
               "(largest residual %.3e)",
               st.unconverged, (long long)(reps * CHUNK_STEPS), units, st.resid_max);
      return fail(c, LBE_ENOCONV, buf);
    }
    t += reps * CHUNK_STEPS;
  }
  for (; t < nsteps; ++t)
    if ((rc = one_step(c))) return rc;
  return LBE_OK;
}

int lbe_record(lbe_ctx *c, int64_t nsteps, int32_t every) {
  if (!c || nsteps < 0 || every < 1)
    return fail(c, LBE_EINVAL, "bad context, step count or checkpoint interval");
  lbe_ctx::Tape &T = c->tape;
  T.t0 = -1;
  const size_t bytes = checkpoint_layout(c).bytes;
  const int64_t nck = (nsteps + every - 1) / every;
  if (nck + 1 > (int64_t)INT32_MAX) return fail(c, LBE_EINVAL, "too many checkpoints");
  if (T.cap < nck + 1) {
    if (T.ck) (void)hipFree(T.ck);
    T.ck = nullptr;
    T.cap = 0;
    int rc = dalloc(c, &T.ck, (size_t)(nck + 1) * bytes);
    if (rc) return rc;
    T.cap = (int)(nck + 1);
  }
  T.hist.assign((size_t)nck + 1, 0);
  for (int64_t t = 0; t < nsteps; ++t) {
    int rc;
    if (t % every == 0) {
      T.hist[(size_t)(t / every)] = c->extrap_hist;
      if ((rc = save_state(c, T.ck + (size_t)(t / every) * bytes))) return rc;
    }
    if ((rc = one_step(c))) return rc;
  }
  T.hist[(size_t)nck] = c->extrap_hist;
  int rc = save_state(c, T.ck + (size_t)nck * bytes);
  if (rc) return rc;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  T.t0 = c->step - nsteps;
  T.nsteps = nsteps;
  T.every = every;
  T.nck = (int)nck;
  return LBE_OK;
}

int lbe_adjoint(lbe_ctx *c, const double *qbar, const double *ubar, double *grad_phi_s,
                double *grad_lB, double *grad_n, double *grad_f) {
  if (!c || (!qbar && !ubar)) return fail(c, LBE_EINVAL, "bad arguments");
  lbe_ctx::Tape &T = c->tape;
  if (T.t0 < 0) return fail(c, LBE_EINVAL, "no recorded steps (lbe_record)");
  if (c->step != T.t0 + T.nsteps || c->qlen < 1)
    return fail(c, LBE_EINVAL, "the state is not the end of the recorded steps");
  if (c->ne == 0 && !ubar) return fail(c, LBE_EINVAL, "no electrode charge to differentiate");
  if (!(c->p.lB > 0.0)) return fail(c, LBE_EINVAL, "reverse mode needs l_B > 0");
  std::vector<double> qb(std::max(c->ne, 1), 0.0), ub(3, 0.0);
  for (int e = 0; e < c->ne && qbar; ++e) qb[e] = qbar[e];
  for (int a = 0; a < 3 && ubar; ++a) ub[a] = ubar[a];
  for (double v : qb)
    if (!std::isfinite(v)) return fail(c, LBE_EINVAL, "non-finite charge weight");
  for (double v : ub)
    if (!std::isfinite(v)) return fail(c, LBE_EINVAL, "non-finite momentum weight");
  int rc = adjoint_buffers(c);
  if (rc) return rc;
  HIPCHK(c, hipMemcpyAsync(c->src_keep, c->src, sizeof(double) * c->L.n, hipMemcpyDeviceToDevice,
                           c->stream));
  const int keep_iters = c->last_iters, keep_pred = c->pred_iters;
  const double keep_resid = c->last_resid;
  const int64_t keep_total = c->total_iters;
  rc = c->mixed ? adjoint_sweep<float>(c, qb.data(), ub.data(), grad_phi_s, grad_lB, grad_n, grad_f)
                : adjoint_sweep<double>(c, qb.data(), ub.data(), grad_phi_s, grad_lB, grad_n, grad_f);
  // back to the end of the recorded steps, whatever happened
  const int rc2 = load_state(c, T.ck + (size_t)T.nck * checkpoint_layout(c).bytes);
  c->extrap_hist = T.hist[(size_t)T.nck];
  if (rc2 == LBE_OK)
    (void)hipMemcpyAsync(c->src, c->src_keep, sizeof(double) * c->L.n, hipMemcpyDeviceToDevice,
                         c->stream);
  (void)hipStreamSynchronize(c->stream);
  c->last_iters = keep_iters;
  c->pred_iters = keep_pred;
  c->last_resid = keep_resid;
  c->total_iters = keep_total;
  return rc ? rc : rc2;
}

int lbe_poisson(lbe_ctx *c, int32_t *iters, double *resid) {
  if (!c) return fail(c, LBE_EINVAL, "context is NULL");
  int rc = poisson_solve(c, false);
  if (iters) *iters = c->last_iters;
  if (resid) *resid = c->last_resid;
  return rc;
}

int lbe_set_electrode_potential(lbe_ctx *c, const double *phi_s) {
  if (!c || !phi_s) return fail(c, LBE_EINVAL, "bad arguments");
  if (!c->solid_idx) {
    for (size_t r = 0; r < c->type_h.size(); ++r)
      if (c->type_h[r]) c->solid_h.push_back((int)r);
    if (c->solid_h.empty()) return LBE_OK;  // no electrode: nothing to set
    HIPCHK(c, hipMalloc((void **)&c->solid_idx, sizeof(int) * c->solid_h.size()));
    HIPCHK(c, hipMalloc((void **)&c->solid_val, sizeof(double) * c->solid_h.size()));
    HIPCHK(c, hipMemcpy(c->solid_idx, c->solid_h.data(), sizeof(int) * c->solid_h.size(),
                        hipMemcpyHostToDevice));
  }
  const size_t S = c->solid_h.size();
  std::vector<double> val(S);
  for (size_t j = 0; j < S; ++j) {
    val[j] = phi_s[c->solid_h[j]];
    if (!std::isfinite(val[j])) return fail(c, LBE_EINVAL, "non-finite electrode potential");
  }
  HIPCHK(c, hipMemcpyAsync(c->solid_val, val.data(), sizeof(double) * S, hipMemcpyHostToDevice,
                           c->stream));
  c->tape.t0 = -1;  // a record of earlier potentials no longer matches the state
  HIPCHK(c, launch_scatter(c->stream, (int)S, c->solid_idx, c->solid_val, c->phi));
  HIPCHK(c, hipStreamSynchronize(c->stream));  // val leaves scope
  int rc = poisson_solve(c, false);
  if (rc) return rc;
  c->extrap_hist = 0;  // the earlier potentials belong to other electrode values
  if (c->ne && c->qlen > 0) {
    rc = charges_to(c, c->qhist + (c->qlen - 1) * c->ne);
    if (rc) return rc;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LBE_OK;
}

int lbe_electrode_charge(lbe_ctx *c, double *q, int32_t ne) {
  if (!c || (!q && ne > 0)) return fail(c, LBE_EINVAL, "bad arguments");
  if (ne < c->ne) return fail(c, LBE_EINVAL, "q has room for fewer values than electrodes");
  if (c->ne == 0) return LBE_OK;
  int rc = charges_to(c, c->qcur);
  if (rc) return rc;
  HIPCHK(c, hipMemcpyAsync(q, c->qcur, sizeof(double) * c->ne, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LBE_OK;
}

int lbe_observables(lbe_ctx *c, lbe_obs *totals, double *phi, double *n, double *u, double *f,
                    double *q_hist, int64_t q_hist_cap, int64_t *q_hist_len) {
  if (!c) return fail(c, LBE_EINVAL, "context is NULL");
  const int K = c->K;
  int rc;
  if (totals) {
    rc = run(c, KK_TOTALS, c->L.n, [&] {
      if (c->mixed)
        return launch_totals_f32(c->stream, c->L, c->P, c->mask, c->h32[c->cur], c->nu32[c->cur],
                                 c->lo32[c->cur], c->partial, c->dout);
      return launch_totals_f64(c->stream, c->L, K, c->p.z, c->mask, c->f[c->cur], c->n[c->cur],
                               c->partial, c->dout);
    });
    if (rc) return rc;
    // total fluid momentum from the pre-collision populations and the Guo
    // velocity of the current state (the observables kernel's output buffers
    // are free between steps)
    const size_t N = (size_t)c->L.n;
    double *fpre = c->mixed ? c->obs : c->f[1 - c->cur];
    double *uo = c->mixed ? c->obs + (size_t)NQ * N : c->u;
    rc = run(c, KK_OBSERVE, c->L.n, [&] {
      if (c->mixed)
        return launch_observe_f32(c->stream, c->L, c->P, c->mask, c->phi, c->nu32[c->cur],
                                  c->h32[c->cur], fpre, uo);
      return launch_observe_f64(c->stream, c->L, c->P, c->mask, c->phi, c->n[c->cur],
                                c->f[c->cur], fpre, uo);
    });
    if (rc) return rc;
    rc = run(c, KK_MOMENTUM, c->L.n, [&] {
      return launch_momentum(c->stream, c->L, c->mask, fpre, uo, c->partial, c->dout + 8);
    });
    if (rc) return rc;
    rc = read_scalars(c, 11);
    if (rc) return rc;
    memset(totals, 0, sizeof *totals);
    totals->step = c->step;
    totals->nelectrodes = c->ne;
    totals->poisson_iters = c->last_iters;
    totals->poisson_resid = c->last_resid;
    totals->mass = c->hpin[0];
    totals->q_ion = c->hpin[1];
    for (int k = 0; k < K; ++k) totals->nk[k] = c->hpin[2 + k];
    totals->poisson_total = c->total_iters;
    for (int a = 0; a < 3; ++a) totals->momentum[a] = c->hpin[8 + a];
  }
  rc = copy_fields(c, phi, n, u, f, hipMemcpyDeviceToHost);
  if (rc) return rc;
  if (q_hist && q_hist_cap > 0 && c->ne > 0) {
    const int64_t rows = std::min(q_hist_cap, c->qlen);
    HIPCHK(c, hipMemcpyAsync(q_hist, c->qhist, sizeof(double) * rows * c->ne, hipMemcpyDeviceToHost,
                             c->stream));
  }
  if (q_hist_len) *q_hist_len = c->qlen;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LBE_OK;
}

void lbe_destroy(lbe_ctx *c) { free_ctx(c); }

int lbe_profile(lbe_ctx *c, int enable) {
  if (!c) return fail(c, LBE_EINVAL, "context is NULL");
  int rc = flush_profile(c);
  if (rc) return rc;
  for (int k = 0; k < KK_COUNT; ++k) {
    c->ms[k] = 0.0;
    c->launches[k] = 0;
    c->units[k] = 0;
  }
  c->prof = enable != 0;
  return LBE_OK;
}

int lbe_kernel_times(lbe_ctx *c, double *ms, int64_t *launches, int64_t *cells, int32_t nkinds) {
  if (!c) return fail(c, LBE_EINVAL, "context is NULL");
  int rc = flush_profile(c);
  if (rc) return rc;
  for (int k = 0; k < nkinds && k < KK_COUNT; ++k) {
    if (ms) ms[k] = c->ms[k];
    if (launches) launches[k] = c->launches[k];
    if (cells) cells[k] = c->units[k];
  }
  return LBE_OK;
}

}  // extern "C"
