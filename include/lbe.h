/*
 * lbe.h -- C ABI of the MI355X (gfx950) Lattice Boltzmann Electrokinetics
 * library: one time step of the LBE method with metallic electrodes of
 * Asta, Palaia, Trizac, Levesque and Rotenberg, "Lattice Boltzmann
 * Electrokinetics simulation of nanocapacitors" (arXiv:1907.04732).
 *
 * Units are lattice units: dx = dt = k_B T = e = 1; phi is the reduced
 * potential beta e psi (Sec. II C); the permittivity is 1/(4 pi l_B).
 *
 * Site order everywhere: r = x + nx*(y + ny*z), x fastest, periodic wrap in
 * all three directions.  Node types: 0 = fluid, e >= 1 = solid node of
 * electrode e (1..LBE_MAX_ELECTRODES).
 *
 * D3Q19 velocity order (populations in lbe_observables and f_init):
 *   0 ( 0, 0, 0)
 *   1 (+1, 0, 0)  2 (-1, 0, 0)  3 ( 0,+1, 0)  4 ( 0,-1, 0)  5 ( 0, 0,+1)  6 ( 0, 0,-1)
 *   7 (+1,+1, 0)  8 (-1,-1, 0)  9 (+1,-1, 0) 10 (-1,+1, 0)
 *  11 (+1, 0,+1) 12 (-1, 0,-1) 13 (+1, 0,-1) 14 (-1, 0,+1)
 *  15 ( 0,+1,+1) 16 ( 0,-1,-1) 17 ( 0,+1,-1) 18 ( 0,-1,+1)
 * weights 1/3 (rest), 1/18 (nearest), 1/36 (next-nearest)  (Sec. II B).
 *
 * Ownership: every host array passed in is copied during the call; the
 * library keeps no host pointer.  The library owns all device memory and
 * frees it in lbe_destroy.  Output pointers are caller-allocated host
 * buffers.  A context is bound to one HIP stream and one device and is not
 * thread-safe; separate contexts are independent.
 *
 * Errors: every int-returning call returns LBE_OK (0) or a negative code;
 * lbe_last_error(ctx) describes the last failure of that context.
 */
#ifndef LBE_H
#define LBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LBE_OK = 0,
  LBE_EINVAL = -1,     /* bad parameter, dimension, pointer or non-finite input */
  LBE_EGEOM = -2,      /* geometry the solver cannot handle (see lbe_init) */
  LBE_ENOMEM = -3,     /* host or device allocation failed */
  LBE_EDEVICE = -4,    /* HIP runtime error, or no gfx950 device */
  LBE_ENOCONV = -5,    /* Poisson solve hit max_iter before tol */
  LBE_ENONFINITE = -6  /* a NaN/Inf appeared in the Poisson residual */
};

enum { LBE_FP64 = 0, LBE_FP32_MIXED = 1 };   /* precision form */
enum { LBE_SOR4 = 0, LBE_MG = 1 };           /* Poisson solver */
enum { LBE_MG_JACOBI = 0, LBE_MG_GS4 = 1 };  /* multigrid smoother */
enum { LBE_ALLOW_FLOATING = 1, LBE_EXTRAPOLATE = 2, LBE_NAIVE_DIRICHLET = 4,
       LBE_KRYLOV = 8 };  /* flags */
enum { LBE_MAX_SPECIES = 4, LBE_MAX_ELECTRODES = 255, LBE_MAX_SITES = 100000000,
       LBE_MAX_SYSTEMS = 8192, LBE_NOALLOC_MAX_ELECTRODES = 16 };

typedef struct lbe_ctx lbe_ctx;

typedef struct {
  int32_t nx, ny, nz;   /* lattice size, each >= 1 */
  int32_t nspecies;     /* 1..4 ionic species */
  int32_t z[4];         /* valencies z_k */
  double D[4];          /* diffusion coefficients D_k >= 0 (Eqs. 9-10) */
  double lB;            /* Bjerrum length l_B >= 0 */
  double tau;           /* BGK relaxation time, > 1/2; nu = (tau - 1/2)/3 */
  double rho0;          /* fluid density of the rest state, > 0 */
  double Eapp[3];       /* applied field beta e E dx (Sec. III A 4) */
  double omega;         /* SOR relaxation factor in (0, 2), diagonal-normalised */
  double tol;           /* Poisson stop: ||R||_inf <= tol; tol <= 0: exactly
                           max_iter sweeps (or cycles) and no LBE_ENOCONV */
  int32_t max_iter;     /* sweep (SOR) or cycle (MG) limit per solve, >= 0 */
  int32_t check_every;  /* sweeps between residual checks, >= 1 */
  int32_t flags;        /* LBE_ALLOW_FLOATING: accept fluid regions that touch
                           no electrode (their mean potential is left free);
                           LBE_EXTRAPOLATE: start each time step's Poisson
                           solve from the quadratic extrapolation in time
                           3 phi(t) - 3 phi(t-1) + phi(t-2) instead of phi(t)
                           (linear on the second step after lbe_init or
                           lbe_set_electrode_potential, phi(t) on the first;
                           same tolerance, fewer iterations);
                           LBE_NAIVE_DIRICHLET: the first-order scheme the
                           paper contrasts with (Sec. II C, Fig. 1): phi_s
                           held on the solid nodes and the plain Laplacian of
                           Eq. 12 (factor 1 on solid-fluid links) in Poisson
                           and in Gauss's law, instead of Eq. 15;
                           LBE_KRYLOV (LBE_MG only, else LBE_EINVAL): each
                           multigrid V-cycle
                           preconditions flexible conjugate gradients (same
                           fixed point and tolerance; fewer cycles where
                           coarse levels represent the electrodes poorly) */
  int32_t precision;    /* LBE_FP64 | LBE_FP32_MIXED */
  int32_t poisson;      /* LBE_SOR4 | LBE_MG */
  int32_t mg_levels;    /* multigrid levels (LBE_MG): 0 = coarsen until at most
                           512 cells remain, whose operator is inverted exactly;
                           else the number of levels (>= 2) */
  int32_t mg_nu1, mg_nu2; /* pre/post smoothing sweeps on the finest level
                           (LBE_MG) */
  int32_t mg_smoother;  /* LBE_MG_JACOBI: undamped Jacobi (smoothing factor 1/2
                           for this stencil, one parallel launch per sweep);
                           LBE_MG_GS4: four-colour Gauss-Seidel */
  int32_t mg_nu1_coarse, mg_nu2_coarse; /* pre/post sweeps on the coarser
                           levels; 0 and 0: the finest level's counts (each
                           launch on a coarse level costs a fixed ~5 us, so
                           one sweep each way there can be the faster cycle) */
  void *stream;         /* hipStream_t to run on; NULL = library-owned stream */
} lbe_params;

typedef struct {
  int64_t step;           /* time steps taken since lbe_init */
  int32_t nelectrodes;    /* largest node type */
  int32_t poisson_iters;  /* sweeps (or cycles) of the last Poisson solve */
  double poisson_resid;   /* ||R||_inf after the last Poisson solve */
  double mass;            /* sum over fluid nodes of rho */
  double nk[4];           /* sum over fluid nodes of n_k */
  double q_ion;           /* sum over fluid nodes of sum_k z_k n_k */
  int64_t poisson_total;  /* sweeps (or cycles) summed over all solves */
  double momentum[3];     /* total fluid momentum sum over fluid nodes of
                             sum_i f_i c_i + F/2 (rho u of Guo forcing), the
                             M of lbe_adjoint; its component along an applied
                             field is the electro-osmotic flux */
} lbe_obs;

/*
 * Create a context and bring it to time 0 (Sec. III A: the uncharged state
 * right after the voltage is applied): populations f_init (19*N, order
 * above; NULL = rest state w_i rho0 on fluid nodes), concentrations n_init
 * (nspecies*N, species-major; NULL = n_ref[k] on every fluid node; values on
 * solid nodes are ignored and set to 0), potential phi_s on solid nodes
 * (N values, fluid entries ignored).  Then solves Poisson for n(0) starting
 * from phi = 0 on fluid nodes and records Q(0).
 *
 * Errors: LBE_EINVAL for tau <= 1/2, omega outside (0, 2), a dimension < 1,
 * more than LBE_MAX_SITES sites,
 * nspecies outside 1..4, negative or non-finite D, l_B < 0, rho0 <= 0,
 * check_every < 1, more than LBE_MAX_ELECTRODES electrodes, a NaN/Inf in any
 * input, or NULL type/phi_s/out; LBE_EGEOM when two neighbouring fluid nodes
 * share a four-colour class (a periodic fluid extent that is odd and > 2
 * along an axis) or when a fluid region touches no electrode and
 * LBE_ALLOW_FLOATING is not set; LBE_EDEVICE without a usable device;
 * LBE_ENOCONV / LBE_ENONFINITE from the first solve (no context is made).
 */
int lbe_init(const lbe_params *params, const uint8_t *type, const double *phi_s,
             const double *n_init, const double *n_ref, const double *f_init, lbe_ctx **out);

/*
 * lbe_init with its arrays in device memory of the current device (for
 * callers whose inputs already live on the GPU, e.g. framework tensors):
 * type (N bytes), phi_s (N), n_init (nspecies*N, may be NULL), n_ref
 * (nspecies, may be NULL) and f_init (19*N, may be NULL), in the layouts of
 * lbe_init.  The arrays are borrowed for the call only: they are read on
 * params->stream (the null stream when NULL), so work that writes them must
 * be ordered before that stream, and the call returns once they are no
 * longer needed.  The geometry is analysed on the host as in lbe_init.
 * Errors: those of lbe_init, plus LBE_EINVAL when a non-NULL array is not
 * device memory of the current device (nothing is read from it), and
 * LBE_EDEVICE when a copy fails.
 */
int lbe_init_device(const lbe_params *params, const uint8_t *type, const double *phi_s,
                    const double *n_init, const double *n_ref, const double *f_init,
                    lbe_ctx **out);

/*
 * Many independent systems in one context (the parameter sweeps of Sec. III:
 * plates of several widths, Debye lengths and voltages).  The systems share
 * one lattice, each enclosed by its own electrodes, and every kernel launch
 * advances all of them.  system[r] (N values, host) is the index
 * 0..nsys-1 of the system a fluid node belongs to (solid entries ignored);
 * no fluid-fluid link may join two systems.  n_ref holds nsys*nspecies
 * values, system-major: the default initial concentrations of each system
 * and, in LBE_FP32_MIXED, the reference of its deviation storage (so each
 * system keeps FP32's relative precision whatever its salt concentration);
 * NULL = each system's fluid mean of n_init.  Populations start at rest.
 * Electrode charges, the Poisson tolerance and all outputs are those of
 * lbe_init for the whole lattice (one electrode id per electrode, up to
 * LBE_MAX_ELECTRODES in total).
 * Errors: as lbe_init, plus LBE_EINVAL for NULL system, nsys outside
 * 1..LBE_MAX_SYSTEMS or an index >= nsys, and LBE_EGEOM when a fluid link
 * joins two systems.
 */
int lbe_init_batch(const lbe_params *params, const uint8_t *type, const double *phi_s,
                   const double *n_init, const double *n_ref, const uint16_t *system,
                   int32_t nsys, lbe_ctx **out);

/*
 * Advance nsteps time steps (Sec. II B-C).  Each step: link fluxes (Eq. 10)
 * and the electrostatic force on the fluid, the velocity u(t); ions
 * n(t+1) = n(t) - sum of link fluxes (Eq. 9); BGK collision with the force
 * and streaming with halfway bounce-back (Eq. 8); Poisson for n(t+1) with
 * the mid-link Dirichlet Laplacian (Eqs. 13, 15), warm-started; the
 * electrode charges Q(t+1) by Gauss's law (Eq. 16) appended to the history.
 * On LBE_ENOCONV / LBE_ENONFINITE the call stops at the failing step and
 * the context goes back to its start: n, f, phi, the step count and the
 * charge history are those of time t (steps completed before it in the same
 * call are kept), and lbe_observables' poisson_iters and poisson_resid
 * report the failed solve.  Under LBE_EXTRAPOLATE the retried step starts
 * from a linear extrapolation (phi(t-2) is not kept).  lbe_set_solver can
 * raise the iteration limit or the tolerance before stepping again.
 */
int lbe_step(lbe_ctx *ctx, int64_t nsteps);

/*
 * Advance nsteps time steps (Sec. II B-C) as lbe_step does, with the steps launched from
 * graphs instead of one by one: 16 whole steps (both passes, the Poisson
 * solve, the electrode charges) are captured once as a HIP graph and
 * replayed, and the host does not wait between steps.  Each replayed step
 * queues the solve's first residual check and then exactly `units` solver
 * units (check_every SOR sweeps, or one multigrid cycle, each ending in a
 * check); a unit that starts after the tolerance was met does nothing on
 * the device, so a step whose solve converges within `units` units gives
 * the same bits as lbe_step.  The steps right after lbe_init or
 * lbe_set_electrode_potential (under LBE_EXTRAPOLATE, until two earlier
 * potentials are kept) and the last nsteps mod 16 run as in lbe_step, as
 * do all steps while per-kernel profiling is on or graphs are disabled.
 * The graph is kept by the context and captured again when units, the
 * tolerance or the buffer parity differ from the last call.
 * The call waits once, after the last replay.  Errors: LBE_EINVAL for
 * nsteps < 0, units < 1, tol <= 0 or units x (iterations per unit) above
 * max_iter; LBE_ENOMEM; LBE_ENOCONV when a replayed step's solve ended
 * above the tolerance, LBE_ENONFINITE when its residual was not finite:
 * unlike lbe_step these are reported after all replays, the context is not
 * rewound, and the state is that after every replayed step (an
 * unconverged step's charges are those of its last iterate; the remaining
 * nsteps mod 16 steps are not taken); lbe_observables' poisson_iters and
 * poisson_resid report the last replayed step.  Otherwise the errors of
 * lbe_step.
 */
int lbe_step_chunk(lbe_ctx *ctx, int64_t nsteps, int32_t units);

/*
 * Change the Poisson stopping rule of a context (the tol and max_iter of
 * lbe_params; the iteration of Sec. II C, Eq. 13) for every later solve: tol <= 0 runs exactly max_iter sweeps
 * (or cycles).  Nothing else changes, so a step that failed with
 * LBE_ENOCONV can be retried with a larger limit.
 * Errors: LBE_EINVAL for a non-finite tol or max_iter < 0 (nothing changed).
 */
int lbe_set_solver(lbe_ctx *ctx, double tol, int32_t max_iter);

/* Re-solve Poisson for the current concentrations, warm-started from the
 * current potential (Sec. II C).  iters/resid may be NULL. */
int lbe_poisson(lbe_ctx *ctx, int32_t *iters, double *resid);

/*
 * New electrode potentials, for time-dependent or non-linear voltage studies
 * (Sec. I and IV name both): phi_s holds N values, of which the solid nodes'
 * are taken (fluid entries ignored, host memory, copied).  Poisson is then
 * re-solved for the current concentrations (warm start from the current
 * potential), and the charge recorded for the current step is replaced by
 * the one of the new potentials, so the history keeps one row per step.
 * Errors: LBE_EINVAL for NULL or a non-finite solid value (nothing changed);
 * LBE_ENOCONV / LBE_ENONFINITE from the solve (the new potentials are kept).
 */
int lbe_set_electrode_potential(lbe_ctx *ctx, const double *phi_s);

/*
 * Reverse mode (gradients of the electrode charge).
 *
 * lbe_record advances nsteps time steps exactly as lbe_step does and keeps,
 * in device memory owned by the context, a checkpoint of the state at the
 * first step and every `every` steps after it, plus the final state:
 * ceil(nsteps/every) + 1 states of (19 + nspecies) N values in the
 * context's storage (8 bytes each in LBE_FP64, 4 in LBE_FP32_MIXED) and N
 * doubles of potential (3 N under LBE_EXTRAPOLATE: the two earlier ones).  It replaces an earlier
 * record.  Errors: LBE_EINVAL for nsteps < 0 or every < 1; LBE_ENOMEM; the
 * errors of lbe_step (then no record is kept).
 *
 * lbe_adjoint returns the gradient of
 *   L = sum_e qbar[e] Q_e(t1) + sum_a ubar[a] M_a(t1),
 * with Q_e the charges of Eq. 16 at the end t1 of the record (qbar:
 * nelectrodes weights, NULL = 0) and M the total fluid momentum
 * sum_r (sum_i f_i c_i + F/2), i.e. the mass flux of the velocity of Guo
 * forcing over all fluid nodes (ubar: 3 weights, NULL = 0; under an applied
 * field its component along the field is the electro-osmotic flux), with
 * respect to
 *   grad_phi_s (N): the potential of every solid node (0 on fluid nodes;
 *     the derivative with respect to one electrode's voltage is the sum
 *     over its nodes);
 *   grad_lB (1 value): the Bjerrum length;
 *   grad_n (nspecies*N): the concentrations at the start t0 of the record;
 *   grad_f (19*N): the pre-collision populations at t0 (the layout of
 *     lbe_init's f_init).
 * Host buffers; any of the four may be NULL.  The derivative is that of the
 * FP64 step, taken backwards along the recorded trajectory (in
 * LBE_FP32_MIXED, the mixed-precision one): streaming and collision
 * (Eq. 8), the link fluxes and the force they exert (Eqs. 9-10), and
 * Poisson (Eqs. 13-15), whose fluid-node operator is symmetric, so each
 * reverse step solves one more Poisson problem with the context's solver,
 * stopped at the same residual tolerance.  The states of one segment between
 * checkpoints are recomputed (one more forward pass in all) and kept as
 * density, momentum, concentrations and potential: min(every, nsteps)
 * states of (5 + nspecies) N doubles (FP32 concentrations in the mixed
 * form), plus (2 (19 + nspecies) + 9) N doubles of adjoint fields.  The
 * context is left at t1, and the record stays valid for further calls with
 * other weights until the state moves (lbe_step, lbe_record,
 * lbe_set_electrode_potential).
 * Errors: LBE_EINVAL for qbar and ubar both NULL, a non-finite weight, no
 * valid record, charge weights without an electrode, or l_B = 0;
 * LBE_ENOMEM; LBE_ENOCONV / LBE_ENONFINITE from a recomputed step or an
 * adjoint solve.
 */
int lbe_record(lbe_ctx *ctx, int64_t nsteps, int32_t every);
int lbe_adjoint(lbe_ctx *ctx, const double *qbar, const double *ubar, double *grad_phi_s,
                double *grad_lB, double *grad_n, double *grad_f);

/* Charge of each electrode, in units of e, from Gauss's law on the current
 * potential (Eq. 16 with the Laplacian of Eq. 15 taken on the electrode's
 * solid nodes, the difference doubled on each solid-fluid link).
 * q has room for ne >= nelectrodes values.  LBE_EINVAL if ne is too small. */
int lbe_electrode_charge(lbe_ctx *ctx, double *q, int32_t ne);

/*
 * lbe_electrode_charge without a context and without allocating, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  The charge of each
 * electrode e = 1..ne from Gauss's law on a potential field, as
 * lbe_electrode_charge computes it (Eq. 16 with the Laplacian of Eq. 15, the
 * difference doubled on each solid-fluid link, or taken once with
 * LBE_NAIVE_DIRICHLET in flags, the only flag accepted):
 *   Q_e = -(6 / 4 pi lB) sum over nodes r of type e of
 *         sum over links i to fluid nodes of wall w_i (phi(r + c_i) - phi(r)).
 * type (N bytes, the node types of lbe_init), phi (N doubles; solid nodes
 * hold their electrode potential) and q (ne doubles, written) are device
 * memory of the current device, in the site order above; nodes of a type
 * above ne are ignored.  The kernels run on `stream` (a hipStream_t; NULL =
 * the null stream) and the call returns without waiting for them.
 * Scratch: the per-block partial sums live in a fixed device array of
 * 256 KiB that the library holds on each GPU it runs on until the process
 * ends; every call on a GPU shares it, so calls that overlap on one GPU
 * (on different streams, or from several threads) race.  Nothing needs
 * clearing between calls.
 * Errors (lbe_last_error(NULL) says which): LBE_EINVAL for a dimension < 1,
 * more than LBE_MAX_SITES sites, ne outside 1..LBE_NOALLOC_MAX_ELECTRODES,
 * lB not finite and > 0, another flag, or a pointer that is NULL or not
 * device memory of the current device (nothing launched); LBE_EDEVICE when
 * the device or a launch fails.
 */
int lbe_electrode_charge_noalloc(int32_t nx, int32_t ny, int32_t nz, double lB, int32_t flags,
                                 const uint8_t *type, const double *phi, double *q, int32_t ne,
                                 void *stream);

/*
 * Copy observables to host buffers (Sec. II B: the moments of the
 * populations and the velocity of Eq. 7; Sec. II C: the electrode charges
 * of Eq. 16); any pointer may be NULL to skip it.
 * totals: lbe_obs; phi: N; n: nspecies*N; u: 3*N component-major (u[a*N+r],
 * the velocity of Guo forcing, (sum_i f_i c_i + F/2)/rho, of the current
 * state); f: 19*N pre-collision populations of the current time; q_hist:
 * up to q_hist_cap rows of nelectrodes charges, Q(0), Q(1), ...;
 * *q_hist_len (if not NULL) receives the number of rows recorded.
 */
int lbe_observables(lbe_ctx *ctx, lbe_obs *totals, double *phi, double *n, double *u,
                    double *f, double *q_hist, int64_t q_hist_cap, int64_t *q_hist_len);

/*
 * The fields of lbe_observables (phi: N; n: nspecies*N; u: 3*N; f: 19*N, in
 * the same layouts, FP64) written into caller-owned device memory of the
 * context's device instead of host memory; any pointer may be NULL.  The
 * copies run on the context's stream and are complete when the call
 * returns.  Errors: LBE_EINVAL when a non-NULL pointer is not device memory
 * of the context's device (nothing written).
 */
int lbe_fields_device(lbe_ctx *ctx, double *phi, double *n, double *u, double *f);

void lbe_destroy(lbe_ctx *ctx);
const char *lbe_strerror(int code);
const char *lbe_last_error(const lbe_ctx *ctx);

/* Kernel timing for the roofline measurement: enable=1 brackets every
 * launch of every kernel kind with HIP events on the context's stream (and
 * launches directly instead of replaying captured graphs); enable=0 stops.
 * Either call clears the counters.  lbe_kernel_times returns, per kind,
 * total milliseconds, launch counts and cells covered (the sum over launches
 * of the cell count of the grid level each launch works on: lattice sites
 * for the finest level) since enabling; it synchronises the stream.  Any of
 * the three host arrays (nkinds entries) may be NULL.  Kinds are listed by
 * lbe_kernel_name. */
int lbe_profile(lbe_ctx *ctx, int enable);
int lbe_kernel_times(lbe_ctx *ctx, double *ms, int64_t *launches, int64_t *cells, int32_t nkinds);
const char *lbe_kernel_name(int32_t kind);
int32_t lbe_num_kernel_kinds(void);

/* Launch shape of the two step passes as the context chose it at init (by
 * timing, or from LBE_PASS_BLOCK / LBE_PASS_TILE): block size of pass A and
 * of pass B (128, 256 or 512; 1 for a pass on LDS-staged tiles of 32 x 8
 * nodes marching along z through runs of 8 planes), and which passes use
 * non-temporal streams (bit 0 pass A, bit 1 pass B).  Any output may be
 * NULL.  Returns LBE_EINVAL for a NULL context. */
int lbe_launch_shape(const lbe_ctx *ctx, int32_t *block_a, int32_t *block_b, int32_t *nontemporal);

/* The D3Q19 velocity set as the library uses it (Sec. II B; 19*3 ints,
 * 19 weights). */
void lbe_velocities(int32_t *c, double *w);

/* Identity of the build: a hash of the sources the library was compiled
 * from (a static string, never NULL; "unknown" when the build did not set
 * it).  A binding compares it with the sources it ships beside, so that a
 * stale library is refused instead of being run. */
const char *lbe_build_id(void);

#ifdef __cplusplus
}
#endif
#endif /* LBE_H */
