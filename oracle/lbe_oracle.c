/*
 * lbe_oracle.c -- plain, slow, FP64 CPU oracle of one Lattice Boltzmann
 * Electrokinetics (LBE) time step with metallic electrodes, after Asta,
 * Palaia, Trizac, Levesque and Rotenberg, "Lattice Boltzmann Electrokinetics
 * simulation of nanocapacitors" (arXiv:1907.04732).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference that the GPU library
 * is checked against.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product path never does.
 * It shares no code, header, table or helper with the GPU library.
 *
 * Everything is double precision, in the order the paper states the method,
 * with no blocking, fusion or reordering.  Built without OpenMP it is single
 * threaded; built with it (only for timing on many cores, and for long test
 * runs) the loops over sites whose iterations are independent run in
 * parallel: one colour of an SOR sweep (no two nodes of a colour are
 * neighbours), the residual maximum, the force, the velocity, the ion update
 * and the LB update (each writes its own site, or, for streaming, a slot no
 * other site writes).  Every value is then bit for bit the single-threaded
 * one; sums over sites (charges, totals) stay serial, in site order.
 *
 *   init : phi <- Poisson(n(0))            (Sec. II C, Eqs. 13 and 15)
 *          Q(0) from Gauss's law             (Sec. II C, Eq. 16)
 *   step : link fluxes, force, velocity u(t) (Sec. II B, Eqs. 7, 9-11)
 *          n(t+1) = n(t) - sum of link fluxes
 *          f(t+1) from BGK collision + streaming with bounce-back (Eq. 8)
 *          phi <- Poisson(n(t+1)), warm start from phi(t)
 *          Q(t+1)
 *
 * This is the per-step order "Poisson(n(t)) -> Q(t) -> fluxes -> n(t+1) ->
 * LB" with the loop rotated so that after every call the potential and the
 * charge belong to the stored concentrations.
 *
 * Readings of places where the paper is silent or its printed formula does
 * not work as written (each is repeated where it is used):
 *   R1 moments are the plain sums rho = sum_i f_i, rho u = sum_i f_i c_i
 *      (the printed w_i weights amount to a rescaling of f_i);
 *   R2 the equilibrium is the usual second-order polynomial in u;
 *   R3 the fluid force keeps only the excess (electrostatic) part of the link
 *      flux, projected on the node with 3 sum_i w_i c_i Delta_i (.), and enters
 *      through Guo forcing (Guo, Zheng and Shi, PRE 65, 046308, 2002);
 *   R4 the link flux carries the prefactor d_k = D_k/A0 and the node update is
 *      n(t+1) - n(t) = -sum_i j_i, which diffuses with coefficient D_k;
 *   R5 advection (deferred by the paper to Capuani et al. 2004) is the central
 *      conservative link flux 3 w_i c_i . (n u(r) + n u(r+c_i));
 *   R6 an applied field enters the ions as a tilt of the excess chemical
 *      potential, delta = z (phi(r') - phi(r) - E . c_i);
 *   R7 the modified Laplacian is applied with the factor 2 on both ends of a
 *      solid-fluid link; solid-solid links carry no charge;
 *   R9 SOR is diagonal-normalised and sweeps four colours in a fixed order.
 *
 * Flag ORC_FLAG_NAIVE_DIRICHLET selects the first-order scheme the paper
 * contrasts with (potential held on the solid nodes, Eq. 12 everywhere).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- error codes (same meaning as the GPU library's) ------------------- */
#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_EGEOM -2
#define ORC_ENOMEM -3
#define ORC_ENOCONV -5
#define ORC_ENONFINITE -6

#define ORC_FLAG_ALLOW_FLOATING 1 /* fluid regions that touch no electrode */
/* The paper's first-order contrast (Sec. II C, before Eq. 14): the electrode
 * potential is held on the solid nodes and the plain Laplacian of Eq. 12 is
 * used on every link (factor 1 instead of 2 on solid-fluid links), both in
 * the Poisson equation and in Gauss's law for the charge. */
#define ORC_FLAG_NAIVE_DIRICHLET 4

/* ---- D3Q19 (Sec. II B): rest, 6 nearest, 12 next-nearest neighbours --- */
#define NQ 19
static const int C[NQ][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static double weight(int i) {
  int n2 = C[i][0] * C[i][0] + C[i][1] * C[i][1] + C[i][2] * C[i][2];
  if (n2 == 0) return 1.0 / 3.0;
  if (n2 == 1) return 1.0 / 18.0;
  return 1.0 / 36.0;
}

/* |c_i| in lattice units (Delta_i of Eq. 10) */
static double link_length(int i) {
  int n2 = C[i][0] * C[i][0] + C[i][1] * C[i][1] + C[i][2] * C[i][2];
  return sqrt((double)n2);
}

/* index of the velocity opposite to c_i */
static int opposite(int i) {
  for (int j = 0; j < NQ; ++j)
    if (C[j][0] == -C[i][0] && C[j][1] == -C[i][1] && C[j][2] == -C[i][2])
      return j;
  return -1;
}

/* ---- parameters and state --------------------------------------------- */
typedef struct {
  int32_t nx, ny, nz, nspecies;
  int32_t z[4];
  double D[4];
  double lB, tau, rho0;
  double Eapp[3];
  double omega, tol;
  int32_t max_iter, check_every;
  int32_t flags, reserved;
} orc_params;

typedef struct {
  orc_params p;
  long N;
  long *nb; /* nb[i*N + r] = periodic neighbour r + c_i */
  int ne;   /* number of electrodes = largest node type */
  unsigned char *type;
  double *phi_s;
  double *phi;
  double *phi_keep; /* phi(t) while step t runs: restored if its solve fails */
  double *n;     /* nspecies * N */
  double *f;     /* NQ * N, pre-collision populations f_i(r, t) */
  double *fnew;  /* NQ * N */
  double *nnew;  /* nspecies * N */
  double *force; /* 3 * N */
  double *u;     /* 3 * N */
  long step;
  int last_iters;
  double last_resid;
  double *qhist; /* ne values per recorded time */
  long qlen, qcap;
  char err[256];
} orc_state;

static long site(const orc_params *p, int x, int y, int z) {
  return (long)x + (long)p->nx * ((long)y + (long)p->ny * (long)z);
}

/* periodic neighbour r + c_i, computed from coordinates */
static long neighbour_of(const orc_params *p, long r, int i) {
  int x = (int)(r % p->nx);
  int y = (int)((r / p->nx) % p->ny);
  int z = (int)(r / ((long)p->nx * p->ny));
  x = (x + C[i][0] + p->nx) % p->nx;
  y = (y + C[i][1] + p->ny) % p->ny;
  z = (z + C[i][2] + p->nz) % p->nz;
  return site(p, x, y, z);
}

/* colour of a site for the four-colour SOR sweep (reading R9) */
static int colour(const orc_params *p, long r) {
  int x = (int)(r % p->nx);
  int y = (int)((r / p->nx) % p->ny);
  int z = (int)(r / ((long)p->nx * p->ny));
  return ((x + z) & 1) + 2 * ((y + z) & 1);
}

static int is_fluid(const orc_state *s, long r) { return s->type[r] == 0; }

/* periodic neighbour r + c_i, looked up in the table filled at init */
static long nbr(const orc_state *s, long r, int i) { return s->nb[(long)i * s->N + r]; }

/* ---- electrostatics (Sec. II C) ---------------------------------------- */

/* Charge density rho_el / e at a node: sum_k z_k n_k (Eq. 2). */
static double charge_density(const orc_state *s, long r) {
  double q = 0.0;
  for (int k = 0; k < s->p.nspecies; ++k) q += s->p.z[k] * s->n[(long)k * s->N + r];
  return q;
}

/*
 * Modified lattice Laplacian at a FLUID node (Eq. 15): the LB-consistent
 * stencil (2/c_s^2) sum_i w_i [phi(r+c_i) - phi(r)] of Eq. 12, with the
 * difference doubled on every link to a solid node, which places the
 * Dirichlet value phi_s at the mid-link.  A link from a node to itself (a box
 * of size 1 along an axis) has a zero difference and is left out.
 */
/* Factor on a solid-fluid link: 2 (Eq. 15), or 1 in the naive mode (Eq. 12). */
static double wall_factor(const orc_state *s) {
  return (s->p.flags & ORC_FLAG_NAIVE_DIRICHLET) ? 1.0 : 2.0;
}

static double laplacian_fluid(const orc_state *s, long r) {
  double acc = 0.0;
  for (int i = 1; i < NQ; ++i) {
    long rn = nbr(s, r, i);
    if (rn == r) continue;
    double factor = is_fluid(s, rn) ? 1.0 : wall_factor(s);
    acc += weight(i) * factor * (s->phi[rn] - s->phi[r]);
  }
  return 6.0 * acc; /* 2 / c_s^2 = 6 */
}

/* Poisson residual R = L_h phi + 4 pi l_B rho_el / e at a fluid node. */
static double residual_at(const orc_state *s, long r) {
  return laplacian_fluid(s, r) + 4.0 * M_PI * s->p.lB * charge_density(s, r);
}

/* max of a and b that keeps a NaN once one has appeared */
static double max_keep_nan(double m, double a) {
  if (m != m) return m;
  return (a != a || a > m) ? a : m;
}

static double residual_inf(const orc_state *s) {
  double m = 0.0;
#pragma omp parallel
  {
    double mt = 0.0;
#pragma omp for schedule(static) nowait
    for (long r = 0; r < s->N; ++r) {
      if (!is_fluid(s, r)) continue;
      mt = max_keep_nan(mt, fabs(residual_at(s, r)));
    }
#pragma omp critical
    m = max_keep_nan(m, mt);
  }
  return m;
}

/*
 * One SOR update of a fluid node (Eq. 13 with the Laplacian of Eq. 15),
 * written in diagonal-normalised form: the Gauss-Seidel value
 *   phi_GS = [sum_i w_i s_i phi(r+c_i) + (4 pi l_B / 6) rho_el] / sum_i w_i s_i
 * (s_i = 2 on links to solid, 1 otherwise) zeroes the residual at r, and
 *   phi <- (1 - omega) phi + omega phi_GS.
 */
static void sor_update(orc_state *s, long r) {
  double num = 0.0, den = 0.0;
  for (int i = 1; i < NQ; ++i) {
    long rn = nbr(s, r, i);
    if (rn == r) continue;
    double ws = weight(i) * (is_fluid(s, rn) ? 1.0 : wall_factor(s));
    num += ws * s->phi[rn];
    den += ws;
  }
  num += 4.0 * M_PI * s->p.lB / 6.0 * charge_density(s, r);
  double gs = num / den;
  s->phi[r] = (1.0 - s->p.omega) * s->phi[r] + s->p.omega * gs;
}

/* One SOR sweep: the four colour classes in order 0, 1, 2, 3. */
static void sor_sweep(orc_state *s) {
  for (int c = 0; c < 4; ++c)
#pragma omp parallel for schedule(static)
    for (long r = 0; r < s->N; ++r)
      if (is_fluid(s, r) && colour(&s->p, r) == c) sor_update(s, r);
}

/*
 * Poisson solve, warm-started from the current phi (Sec. II C).  The residual
 * infinity-norm is taken before the first sweep and after every check_every
 * sweeps; the solve stops when it is <= tol.  tol <= 0 means "exactly
 * max_iter sweeps" (used to compare iterates), with no convergence error.
 */
static int poisson_solve(orc_state *s) {
  const orc_params *p = &s->p;
  int sweeps = 0;
  if (p->tol <= 0.0) {
    for (sweeps = 0; sweeps < p->max_iter; ++sweeps) sor_sweep(s);
    s->last_iters = sweeps;
    s->last_resid = residual_inf(s);
    if (!isfinite(s->last_resid)) return ORC_ENONFINITE;
    return ORC_OK;
  }
  for (;;) {
    double res = residual_inf(s);
    s->last_iters = sweeps;
    s->last_resid = res;
    if (!isfinite(res)) {
      snprintf(s->err, sizeof s->err, "non-finite Poisson residual");
      return ORC_ENONFINITE;
    }
    if (res <= p->tol) return ORC_OK;
    if (sweeps >= p->max_iter) {
      snprintf(s->err, sizeof s->err,
               "Poisson not converged: residual %.3e after %d sweeps", res, sweeps);
      return ORC_ENOCONV;
    }
    for (int m = 0; m < p->check_every && sweeps < p->max_iter; ++m, ++sweeps)
      sor_sweep(s);
  }
}

/*
 * Charge of each electrode from Gauss's law (Eq. 16):
 *   Q_e = -(1 / 4 pi l_B) sum_{r in e} L_h phi(r),
 * with L_h evaluated at the electrode's solid nodes by Eq. 15.  The printed
 * factor [1 + chi(r') - chi(r)] vanishes on a solid-to-fluid link, which would
 * make Q identically zero; the factor 2 is taken on both ends of each
 * solid-fluid link (reading R7), and solid-solid links (inside an electrode or
 * between two electrodes) carry nothing.  q[e-1] is in units of e.
 */
static void electrode_charges(const orc_state *s, double *q) {
  for (int e = 0; e < s->ne; ++e) q[e] = 0.0;
  for (long r = 0; r < s->N; ++r) {
    int e = s->type[r];
    if (e == 0) continue;
    double lap = 0.0;
    for (int i = 1; i < NQ; ++i) {
      long rn = nbr(s, r, i);
      if (!is_fluid(s, rn)) continue;
      lap += weight(i) * wall_factor(s) * (s->phi[rn] - s->phi[r]);
    }
    q[e - 1] += -(6.0 * lap) / (4.0 * M_PI * s->p.lB);
  }
}

static int record_charge(orc_state *s) {
  if (s->qlen == s->qcap) {
    long cap = s->qcap ? 2 * s->qcap : 1024;
    double *nq = (double *)realloc(s->qhist, sizeof(double) * (size_t)cap * (size_t)(s->ne ? s->ne : 1));
    if (!nq) return ORC_ENOMEM;
    s->qhist = nq;
    s->qcap = cap;
  }
  if (s->ne) electrode_charges(s, s->qhist + s->qlen * s->ne);
  s->qlen++;
  return ORC_OK;
}

/* ---- ions and fluid (Sec. II B) ---------------------------------------- */

#define A0 (1.0 + 2.0 * M_SQRT2) /* lattice factor of Eq. 9 for D3Q19 */

/*
 * Excess part of the link flux (Eq. 10) of species k on the link r -> r':
 * the symmetrised flux -d_k (e^{-mu} + e^{-mu'})/2 (n' e^{mu'} - n e^{mu})/Delta
 * splits exactly into an ideal part -d_k (n' - n)/Delta and
 *   d_k g,   g = -[n' expm1(delta) - n expm1(-delta)] / (2 Delta),
 * with delta = mu'^ex - mu^ex = z (phi' - phi - E . c_i)  (reading R6).
 */
static double excess_link(double n_here, double n_there, double delta, double len) {
  return -(n_there * expm1(delta) - n_here * expm1(-delta)) / (2.0 * len);
}

/* Force density on the fluid at every fluid node (reading R3). */
static void compute_force(orc_state *s) {
  const orc_params *p = &s->p;
#pragma omp parallel for schedule(static)
  for (long r = 0; r < s->N; ++r) {
    double F[3] = {0.0, 0.0, 0.0};
    if (is_fluid(s, r)) {
      for (int i = 1; i < NQ; ++i) {
        long rn = nbr(s, r, i);
        if (!is_fluid(s, rn)) continue; /* no flux through solid links */
        double len = link_length(i);
        double Ec = p->Eapp[0] * C[i][0] + p->Eapp[1] * C[i][1] + p->Eapp[2] * C[i][2];
        double gsum = 0.0;
        for (int k = 0; k < p->nspecies; ++k) {
          double delta = p->z[k] * (s->phi[rn] - s->phi[r] - Ec);
          gsum += excess_link(s->n[(long)k * s->N + r], s->n[(long)k * s->N + rn], delta, len);
        }
        for (int a = 0; a < 3; ++a) F[a] += 3.0 * weight(i) * C[i][a] * len * gsum;
      }
    }
    for (int a = 0; a < 3; ++a) s->force[3 * r + a] = F[a];
  }
}

/* Density and velocity (Eq. 7, reading R1) with the half-force shift of Guo
 * forcing: u = (sum_i f_i c_i + F/2) / rho. */
static void compute_velocity(orc_state *s) {
#pragma omp parallel for schedule(static)
  for (long r = 0; r < s->N; ++r) {
    double rho = 0.0, m[3] = {0.0, 0.0, 0.0};
    if (is_fluid(s, r)) {
      for (int i = 0; i < NQ; ++i) {
        double fi = s->f[(long)i * s->N + r];
        rho += fi;
        for (int a = 0; a < 3; ++a) m[a] += fi * C[i][a];
      }
      for (int a = 0; a < 3; ++a) s->u[3 * r + a] = (m[a] + 0.5 * s->force[3 * r + a]) / rho;
    } else {
      for (int a = 0; a < 3; ++a) s->u[3 * r + a] = 0.0;
    }
  }
}

/*
 * Ion update (Eqs. 9-10, readings R4-R6): for each fluid node and each link
 * to a fluid neighbour, the diffusion-migration flux
 *   j = d_k [g - (n' - n)/Delta],  d_k = D_k / A0,
 * plus the advective flux J = 3 w_i c_i . (n u(r) + n' u(r')), and
 *   n(t+1) = n(t) - sum_i (j + J).
 * Links to solid nodes carry no flux, so no ion enters an electrode.
 */
static void update_ions(orc_state *s) {
  const orc_params *p = &s->p;
  for (int k = 0; k < p->nspecies; ++k) {
    const double *nk = s->n + (long)k * s->N;
    double *out = s->nnew + (long)k * s->N;
    double dk = p->D[k] / A0;
#pragma omp parallel for schedule(static)
    for (long r = 0; r < s->N; ++r) {
      if (!is_fluid(s, r)) {
        out[r] = nk[r];
        continue;
      }
      double sum = 0.0;
      for (int i = 1; i < NQ; ++i) {
        long rn = nbr(s, r, i);
        if (!is_fluid(s, rn)) continue;
        double len = link_length(i);
        double Ec = p->Eapp[0] * C[i][0] + p->Eapp[1] * C[i][1] + p->Eapp[2] * C[i][2];
        double delta = p->z[k] * (s->phi[rn] - s->phi[r] - Ec);
        double g = excess_link(nk[r], nk[rn], delta, len);
        double j = dk * (g - (nk[rn] - nk[r]) / len);
        double cu_here = 0.0, cu_there = 0.0;
        for (int a = 0; a < 3; ++a) {
          cu_here += C[i][a] * s->u[3 * r + a];
          cu_there += C[i][a] * s->u[3 * rn + a];
        }
        double J = 3.0 * weight(i) * (nk[r] * cu_here + nk[rn] * cu_there);
        sum += j + J;
      }
      out[r] = nk[r] - sum;
    }
  }
  double *t = s->n;
  s->n = s->nnew;
  s->nnew = t;
}

/*
 * LB update (Eq. 8): BGK relaxation towards the second-order equilibrium
 * (reading R2) with the Guo forcing term, then streaming.  A population that
 * would enter a solid node is reflected back to its origin with the opposite
 * velocity (halfway bounce-back: the wall sits at the mid-link).
 */
static void update_fluid(orc_state *s) {
  const orc_params *p = &s->p;
  const double tau = p->tau;
#pragma omp parallel for schedule(static)
  for (long r = 0; r < s->N; ++r) {
    if (!is_fluid(s, r)) continue;
    double rho = 0.0;
    for (int i = 0; i < NQ; ++i) rho += s->f[(long)i * s->N + r];
    const double *u = s->u + 3 * r;
    const double *F = s->force + 3 * r;
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < NQ; ++i) {
      double cu = C[i][0] * u[0] + C[i][1] * u[1] + C[i][2] * u[2];
      double feq = weight(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
      double src = 0.0;
      for (int a = 0; a < 3; ++a) src += (3.0 * (C[i][a] - u[a]) + 9.0 * cu * C[i][a]) * F[a];
      src *= (1.0 - 0.5 / tau) * weight(i);
      double fi = s->f[(long)i * s->N + r];
      double post = fi - (fi - feq) / tau + src;
      long rn = nbr(s, r, i);
      if (is_fluid(s, rn))
        s->fnew[(long)i * s->N + rn] = post;
      else
        s->fnew[(long)opposite(i) * s->N + r] = post;
    }
  }
  double *t = s->f;
  s->f = s->fnew;
  s->fnew = t;
}

/* ---- geometry checks ---------------------------------------------------- */

/* The four-colour order needs neighbouring fluid nodes to differ in colour. */
static int check_colouring(const orc_state *s) {
  for (long r = 0; r < s->N; ++r) {
    if (!is_fluid(s, r)) continue;
    for (int i = 1; i < NQ; ++i) {
      long rn = nbr(s, r, i);
      if (rn == r || !is_fluid(s, rn)) continue;
      if (colour(&s->p, rn) == colour(&s->p, r)) return 0;
    }
  }
  return 1;
}

/* Every connected fluid region must touch an electrode, or the Poisson
 * problem on it has no unique solution. */
static int check_connectivity(const orc_state *s) {
  long N = s->N;
  int *label = (int *)malloc(sizeof(int) * (size_t)N);
  long *stack = (long *)malloc(sizeof(long) * (size_t)N);
  if (!label || !stack) {
    free(label);
    free(stack);
    return -1;
  }
  for (long r = 0; r < N; ++r) label[r] = 0;
  int ok = 1;
  for (long r0 = 0; r0 < N && ok; ++r0) {
    if (!is_fluid(s, r0) || label[r0]) continue;
    long top = 0;
    stack[top++] = r0;
    label[r0] = 1;
    int touches = 0;
    while (top) {
      long r = stack[--top];
      for (int i = 1; i < NQ; ++i) {
        long rn = nbr(s, r, i);
        if (!is_fluid(s, rn)) {
          touches = 1;
          continue;
        }
        if (!label[rn]) {
          label[rn] = 1;
          stack[top++] = rn;
        }
      }
    }
    if (!touches) ok = 0;
  }
  free(label);
  free(stack);
  return ok;
}

/* ---- public API --------------------------------------------------------- */

const char *orc_strerror(int code) {
  switch (code) {
    case ORC_OK: return "ok";
    case ORC_EINVAL: return "invalid argument";
    case ORC_EGEOM: return "invalid geometry";
    case ORC_ENOMEM: return "out of memory";
    case ORC_ENOCONV: return "Poisson solve did not converge";
    case ORC_ENONFINITE: return "non-finite value";
    default: return "unknown error";
  }
}

const char *orc_last_error(const orc_state *s) { return s ? s->err : ""; }

void orc_free(orc_state *s) {
  if (!s) return;
  free(s->nb);
  free(s->type);
  free(s->phi_s);
  free(s->phi);
  free(s->phi_keep);
  free(s->n);
  free(s->nnew);
  free(s->f);
  free(s->fnew);
  free(s->force);
  free(s->u);
  free(s->qhist);
  free(s);
}

static int validate(const orc_params *p, char *err, size_t errlen) {
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) {
    snprintf(err, errlen, "lattice dimensions must be >= 1");
    return ORC_EINVAL;
  }
  if (p->nspecies < 1 || p->nspecies > 4) {
    snprintf(err, errlen, "nspecies must be in 1..4");
    return ORC_EINVAL;
  }
  if (!(p->tau > 0.5)) {
    snprintf(err, errlen, "tau must exceed 1/2");
    return ORC_EINVAL;
  }
  if (!(p->omega > 0.0 && p->omega < 2.0)) {
    snprintf(err, errlen, "omega must lie in (0, 2)");
    return ORC_EINVAL;
  }
  if (!(p->rho0 > 0.0) || !(p->lB >= 0.0) || !isfinite(p->tol) || p->max_iter < 0 ||
      p->check_every < 1) {
    snprintf(err, errlen, "bad rho0, lB, tol, max_iter or check_every");
    return ORC_EINVAL;
  }
  for (int k = 0; k < p->nspecies; ++k)
    if (!(p->D[k] >= 0.0) || !isfinite(p->D[k])) {
      snprintf(err, errlen, "diffusion coefficients must be finite and >= 0");
      return ORC_EINVAL;
    }
  for (int a = 0; a < 3; ++a)
    if (!isfinite(p->Eapp[a])) {
      snprintf(err, errlen, "applied field must be finite");
      return ORC_EINVAL;
    }
  if (p->flags & ~(ORC_FLAG_ALLOW_FLOATING | ORC_FLAG_NAIVE_DIRICHLET)) {
    snprintf(err, errlen, "unknown flags");
    return ORC_EINVAL;
  }
  return ORC_OK;
}

/*
 * Build the state.  type[r] = 0 for fluid, e >= 1 for a node of electrode e;
 * phi_s[r] is the potential of solid nodes (fluid entries ignored);
 * n_init (nspecies*N, NULL = n_ref on fluid nodes), f_init (19*N, NULL =
 * rest populations w_i rho0).  Ends with the first Poisson solve and Q(0).
 */
int orc_init(const orc_params *pin, const unsigned char *type, const double *phi_s,
             const double *n_init, const double *n_ref, const double *f_init,
             orc_state **out, char *errbuf, int errlen) {
  char err[256] = "";
  *out = NULL;
  int rc = validate(pin, err, sizeof err);
  if (rc) {
    if (errbuf) snprintf(errbuf, (size_t)errlen, "%s", err);
    return rc;
  }
  orc_state *s = (orc_state *)calloc(1, sizeof(orc_state));
  if (!s) return ORC_ENOMEM;
  s->p = *pin;
  long N = (long)pin->nx * pin->ny * pin->nz;
  int K = pin->nspecies;
  s->N = N;
  s->type = (unsigned char *)malloc((size_t)N);
  s->phi_s = (double *)malloc(sizeof(double) * (size_t)N);
  s->phi = (double *)calloc((size_t)N, sizeof(double));
  s->phi_keep = (double *)calloc((size_t)N, sizeof(double));
  s->n = (double *)calloc((size_t)N * K, sizeof(double));
  s->nnew = (double *)calloc((size_t)N * K, sizeof(double));
  s->f = (double *)calloc((size_t)N * NQ, sizeof(double));
  s->fnew = (double *)calloc((size_t)N * NQ, sizeof(double));
  s->force = (double *)calloc((size_t)N * 3, sizeof(double));
  s->u = (double *)calloc((size_t)N * 3, sizeof(double));
  s->nb = (long *)malloc(sizeof(long) * (size_t)N * NQ);
  if (!s->nb || !s->type || !s->phi_s || !s->phi || !s->n || !s->nnew || !s->f || !s->fnew ||
      !s->force || !s->u) {
    orc_free(s);
    return ORC_ENOMEM;
  }
  memcpy(s->type, type, (size_t)N);
  for (int i = 0; i < NQ; ++i)
    for (long r = 0; r < N; ++r) s->nb[(long)i * N + r] = neighbour_of(pin, r, i);
  s->ne = 0;
  for (long r = 0; r < N; ++r)
    if (type[r] > s->ne) s->ne = type[r];
  for (long r = 0; r < N; ++r) {
    if (type[r]) {
      if (!isfinite(phi_s[r])) {
        snprintf(err, sizeof err, "non-finite electrode potential");
        rc = ORC_EINVAL;
        break;
      }
      s->phi_s[r] = phi_s[r];
      s->phi[r] = phi_s[r];
    } else {
      s->phi_s[r] = 0.0;
      s->phi[r] = 0.0;
    }
  }
  for (int k = 0; k < K && !rc; ++k)
    for (long r = 0; r < N; ++r) {
      double v = 0.0;
      if (type[r] == 0) v = n_init ? n_init[(long)k * N + r] : (n_ref ? n_ref[k] : 0.0);
      if (!isfinite(v)) {
        snprintf(err, sizeof err, "non-finite initial concentration");
        rc = ORC_EINVAL;
        break;
      }
      s->n[(long)k * N + r] = v;
    }
  for (int i = 0; i < NQ && !rc; ++i)
    for (long r = 0; r < N; ++r) {
      double v = 0.0;
      if (type[r] == 0) v = f_init ? f_init[(long)i * N + r] : weight(i) * pin->rho0;
      if (!isfinite(v)) {
        snprintf(err, sizeof err, "non-finite initial population");
        rc = ORC_EINVAL;
        break;
      }
      s->f[(long)i * N + r] = v;
    }
  if (!rc && !check_colouring(s)) {
    snprintf(err, sizeof err,
             "four-colour order invalid: periodic fluid extent along an axis is odd and > 2");
    rc = ORC_EGEOM;
  }
  if (!rc && !(pin->flags & ORC_FLAG_ALLOW_FLOATING)) {
    int c = check_connectivity(s);
    if (c < 0) rc = ORC_ENOMEM;
    else if (!c) {
      snprintf(err, sizeof err, "a fluid region touches no electrode");
      rc = ORC_EGEOM;
    }
  }
  if (!rc) {
    rc = poisson_solve(s);
    if (rc) snprintf(err, sizeof err, "%s", s->err);
  }
  if (!rc) rc = record_charge(s);
  if (rc) {
    if (errbuf) snprintf(errbuf, (size_t)errlen, "%s", err);
    orc_free(s);
    return rc;
  }
  *out = s;
  return ORC_OK;
}

/* Advance nsteps time steps.  When a step's Poisson solve fails, the state
 * (n, f, phi, step count, charge history) goes back to the start of that
 * step and its error code is returned. */
int orc_step(orc_state *s, long nsteps) {
  if (!s || nsteps < 0) return ORC_EINVAL;
  for (long t = 0; t < nsteps; ++t) {
    compute_force(s);
    compute_velocity(s);
    memcpy(s->phi_keep, s->phi, sizeof(double) * (size_t)s->N);
    update_ions(s);
    update_fluid(s);
    s->step++;
    int rc = poisson_solve(s);
    if (rc) {
      /* back to the start of the failing step: the previous n and f are
       * still in the buffers the updates swapped out */
      double *t = s->n;
      s->n = s->nnew;
      s->nnew = t;
      t = s->f;
      s->f = s->fnew;
      s->fnew = t;
      memcpy(s->phi, s->phi_keep, sizeof(double) * (size_t)s->N);
      s->step--;
      return rc;
    }
    rc = record_charge(s);
    if (rc) return rc;
  }
  return ORC_OK;
}

/*
 * New electrode potentials (a time-dependent or non-linear voltage study,
 * Sec. I and IV): phi_s[r] is taken for every solid node (fluid entries are
 * ignored), Poisson is re-solved for the current concentrations (warm start
 * from the current phi), and the charge recorded for the current step is
 * replaced by the one of the new potentials.
 */
int orc_set_electrode_potential(orc_state *s, const double *phi_s) {
  if (!s || !phi_s) return ORC_EINVAL;
  for (long r = 0; r < s->N; ++r)
    if (s->type[r] && !isfinite(phi_s[r])) {
      snprintf(s->err, sizeof s->err, "non-finite electrode potential");
      return ORC_EINVAL;
    }
  for (long r = 0; r < s->N; ++r)
    if (s->type[r]) {
      s->phi_s[r] = phi_s[r];
      s->phi[r] = phi_s[r];
    }
  int rc = poisson_solve(s);
  if (rc) return rc;
  if (s->ne && s->qlen > 0) electrode_charges(s, s->qhist + (s->qlen - 1) * s->ne);
  return ORC_OK;
}

/* Re-solve Poisson for the current concentrations (warm start). */
/* New Poisson stopping rule (tol <= 0: exactly max_iter sweeps). */
int orc_set_solver(orc_state *s, double tol, int max_iter) {
  if (!s || !isfinite(tol) || max_iter < 0) return ORC_EINVAL;
  s->p.tol = tol;
  s->p.max_iter = max_iter;
  return ORC_OK;
}

int orc_poisson(orc_state *s, int *iters, double *resid) {
  int rc = poisson_solve(s);
  if (iters) *iters = s->last_iters;
  if (resid) *resid = s->last_resid;
  return rc;
}

int orc_electrode_charge(const orc_state *s, double *q, int ne) {
  if (!s || ne < s->ne) return ORC_EINVAL;
  electrode_charges(s, q);
  return ORC_OK;
}

int orc_num_electrodes(const orc_state *s) { return s->ne; }
long orc_step_count(const orc_state *s) { return s->step; }
int orc_last_iters(const orc_state *s) { return s->last_iters; }
double orc_last_resid(const orc_state *s) { return s->last_resid; }

/*
 * Copy fields out (NULL = skip): phi (N), n (nspecies*N), pre-collision
 * populations f (19*N), density rho (N) and velocity u (3*N, component-major
 * u[a*N + r]) of the current populations with the current force, and the
 * force density (3*N, component-major).
 */
int orc_fields(orc_state *s, double *phi, double *n, double *f, double *rho, double *u,
               double *force) {
  long N = s->N;
  if (phi) memcpy(phi, s->phi, sizeof(double) * (size_t)N);
  if (n) memcpy(n, s->n, sizeof(double) * (size_t)N * s->p.nspecies);
  if (f) memcpy(f, s->f, sizeof(double) * (size_t)N * NQ);
  if (rho || u || force) {
    compute_force(s);
    compute_velocity(s);
    for (long r = 0; r < N; ++r) {
      double d = 0.0;
      if (is_fluid(s, r))
        for (int i = 0; i < NQ; ++i) d += s->f[(long)i * N + r];
      if (rho) rho[r] = d;
      for (int a = 0; a < 3; ++a) {
        if (u) u[(long)a * N + r] = s->u[3 * r + a];
        if (force) force[(long)a * N + r] = s->force[3 * r + a];
      }
    }
  }
  return ORC_OK;
}

/* Residual field R = L_h phi + 4 pi l_B rho_el on fluid nodes (0 on solid). */
int orc_residual(const orc_state *s, double *res) {
  for (long r = 0; r < s->N; ++r) res[r] = is_fluid(s, r) ? residual_at(s, r) : 0.0;
  return ORC_OK;
}

/* Charge history: qlen entries of ne values each (Q(0), Q(1), ...). */
long orc_qhist(const orc_state *s, double *out, long cap) {
  long m = s->qlen < cap ? s->qlen : cap;
  if (out && s->ne) memcpy(out, s->qhist, sizeof(double) * (size_t)m * s->ne);
  return s->qlen;
}

/* Threads of the parallel loops: sets the count when n > 0 and returns the
 * count in use (1 when built without OpenMP). */
int orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

/* The velocity set, for checking that both implementations agree on it. */
void orc_velocities(int *c /* 19*3 */, double *w /* 19 */) {
  for (int i = 0; i < NQ; ++i) {
    for (int a = 0; a < 3; ++a) c[3 * i + a] = C[i][a];
    w[i] = weight(i);
  }
}
