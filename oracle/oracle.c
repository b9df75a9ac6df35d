/*
 * oracle.c -- plain FP64 CPU reference of the two-body macro-ion PIC step.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Written for clarity, not speed:
 * every shape weight is evaluated from the B-spline definition, every sum
 * is a plain loop, and nothing is blocked, fused or reordered.
 *
 * Paper: An, Chen, Sheng, Zhang, arXiv 2208.08038.
 *   Sec. 2  two-body macro-ion (q2 = -Z_b e, m2 = Z_b m_e, q1 = q_c - q2,
 *           m1 = m_c - m2), Boris update of each body with the internal
 *           force added to E, current q v / dV of each body, initial split
 *           p1 + p2 = p_c with q1 v1 + q2 v2 = 0, softened Coulomb potential
 *           V_M = q1 q2 / (4 pi eps0 sqrt(r^2 + a_c^2)).
 *   Sec. 3.1 restoring frequency w_c^2 = |q1 q2| / (4 pi eps0 m_r a_c^3),
 *           centre of mass r_c, r = r1 - r2, reduced mass m_r.
 * Where the paper is silent (shape, deposition, field solver, boundaries,
 * damping) the readings are: quadratic B-spline shape, Esirkepov
 * charge-conserving deposit, Yee leapfrog, first-order Mur open faces with
 * the laser entering through x-min, reflecting particle walls `pad` cells
 * inside open faces, and a momentum-conserving Crank-Nicolson friction on
 * the relative momentum.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAX_SPECIES 8
#define OR_PI 3.14159265358979323846

#define OR_MAX_SHELL 4

typedef struct {
  int kind;
  double q1, m1, q2, m2; /* real-particle charges and masses (point: q1, m1) */
  /* multi-shell ion: nucleus (q1, m1) and nshell clouds with their own
     charge, mass, bond frequency and softening length */
  int nshell;
  double qk[OR_MAX_SHELL], mk[OR_MAX_SHELL], wk[OR_MAX_SHELL], ak[OR_MAX_SHELL];
  double weight, omega_c, a_c, nu, nu_per_omega;
  int ac_derived;  /* a_c of each ion from its own omega_c (Sec. 3.1) */
  double re_norm;  /* Coulomb constant of the bond in these units */
  int64_t n, cap;
  int32_t* cell; /* n x 3 */
  double* off;   /* n x 3 */
  double* delta; /* n x 3 (multi-shell: n x 3 nshell, shell k at 3k) */
  double* u1;    /* n x 3 */
  double* u2;    /* n x 3 (multi-shell: n x 3 nshell) */
  double* wc;    /* per-particle omega_c or NULL */
  double* w;     /* per-particle weight or NULL */
} or_species;

struct or_ctx {
  or_config g;
  int nd;
  int64_t nn[3]; /* interior cells per dim (1 for unresolved) */
  int64_t st[3]; /* storage extent per dim (n+2 for resolved, 1 otherwise) */
  int64_t gh[3]; /* ghost offset per dim (1 resolved, 0 otherwise) */
  int64_t ntot, ncell;
  double* E[3];
  double* B[3];
  double* J[3];
  double* mur_b[3][2]; /* per dim: tangential B at the first interior node, previous half step */
  double* mur_e[3][2]; /* per dim: tangential E at the last interior node, time n */
  or_species sp[OR_MAX_SPECIES];
  int nsp;
  int64_t step;
  uint32_t err;
  double div_l2, div_max, rho_l2;
  int nprobe;
  int32_t* pcomp;
  int64_t* pidx;
  double* pdata;
  int64_t nrec;
};

/* ---------------------------------------------------------------- helpers */

static int resolved(const or_ctx* c, int d) { return d < c->nd; }
static int periodic(const or_ctx* c, int d) {
  return c->g.bc_lo[d] == OR_PERIODIC && c->g.bc_hi[d] == OR_PERIODIC;
}

static int64_t fidx(const or_ctx* c, int64_t i, int64_t j, int64_t k) {
  return (i + c->gh[0]) + c->st[0] * ((j + c->gh[1]) + c->st[1] * (k + c->gh[2]));
}
static int64_t cidx(const or_ctx* c, int64_t i, int64_t j, int64_t k) {
  return i + c->nn[0] * (j + c->nn[1] * k);
}

/* Map an interior-relative node index along d into [0, n) for periodic
   dimensions.  For open dimensions the index must already be interior;
   returns 0 if it is not. */
static int wrap(const or_ctx* c, int d, int64_t* i) {
  if (!resolved(c, d)) return *i == 0;
  int64_t n = c->nn[d];
  if (periodic(c, d)) {
    *i = ((*i % n) + n) % n;
    return 1;
  }
  return *i >= 0 && *i < n;
}

/* Quadratic B-spline (the order-2 particle shape): 3/4 - d^2 for |d| < 1/2,
   (3/2 - |d|)^2 / 2 for 1/2 <= |d| < 3/2, zero beyond. */
static double b2(double d) {
  double a = fabs(d);
  if (a < 0.5) return 0.75 - a * a;
  if (a < 1.5) {
    double t = 1.5 - a;
    return 0.5 * t * t;
  }
  return 0.0;
}

/* Nodes considered around a particle's cell, relative index -2 .. +3. */
#define RLO (-2)
#define NW 6

/* -------------------------------------------------------------- creation */

or_ctx* or_create(const or_config* cfg) {
  if (!cfg || cfg->ndim < 1 || cfg->ndim > 3) return NULL;
  /* an oblique wave is a plane wave in a resolved x-y plane */
  if (cfg->angle != 0.0 && (cfg->ndim < 2 || cfg->waist > 0.0)) return NULL;
  if (cfg->n_env < 0 || cfg->n_env > OR_MAX_ENV) return NULL;
  or_ctx* c = (or_ctx*)calloc(1, sizeof(or_ctx));
  c->g = *cfg;
  c->nd = cfg->ndim;
  c->ntot = 1;
  c->ncell = 1;
  for (int d = 0; d < 3; d++) {
    if (d < c->nd) {
      if (cfg->n[d] < 1 || !(cfg->dx[d] > 0)) {
        free(c);
        return NULL;
      }
      c->nn[d] = cfg->n[d];
      c->st[d] = cfg->n[d] + 2;
      c->gh[d] = 1;
    } else {
      c->nn[d] = 1;
      c->st[d] = 1;
      c->gh[d] = 0;
    }
    c->ntot *= c->st[d];
    c->ncell *= c->nn[d];
  }
  for (int a = 0; a < 3; a++) {
    c->E[a] = (double*)calloc((size_t)c->ntot, sizeof(double));
    c->B[a] = (double*)calloc((size_t)c->ntot, sizeof(double));
    c->J[a] = (double*)calloc((size_t)c->ntot, sizeof(double));
  }
  for (int d = 0; d < c->nd; d++) {
    int64_t plane = c->ncell / c->nn[d];
    for (int t = 0; t < 2; t++) {
      c->mur_b[d][t] = (double*)calloc((size_t)plane, sizeof(double));
      c->mur_e[d][t] = (double*)calloc((size_t)plane, sizeof(double));
    }
  }
  return c;
}

void or_destroy(or_ctx* c) {
  if (!c) return;
  for (int a = 0; a < 3; a++) {
    free(c->E[a]);
    free(c->B[a]);
    free(c->J[a]);
  }
  for (int d = 0; d < 3; d++)
    for (int t = 0; t < 2; t++) {
      free(c->mur_b[d][t]);
      free(c->mur_e[d][t]);
    }
  for (int s = 0; s < c->nsp; s++) {
    or_species* p = &c->sp[s];
    free(p->cell);
    free(p->off);
    free(p->delta);
    free(p->u1);
    free(p->u2);
    free(p->wc);
    free(p->w);
  }
  free(c->pcomp);
  free(c->pidx);
  free(c->pdata);
  free(c);
}

/* Sec. 3.1: w_c^2 = |q1 q2| / (4 pi eps0 m_r a_c^3).  In the normalised
   units the Coulomb constant e^2/(4 pi eps0) becomes the normalised
   classical electron radius re_norm = 2 pi r_e / lambda (with m_e c^2 = 1). */
double or_ac_from_omega(double q1, double m1, double q2, double m2, double omega_c,
                        double re_norm) {
  double mr = m1 * m2 / (m1 + m2);
  return cbrt(fabs(q1 * q2) * re_norm / (mr * omega_c * omega_c));
}

/* Softening length of the bond: a_c = 0 asks for a_c^3 = |q1 q2| re_norm /
   (m_r omega_c^2) with each ion's own omega_c, because the Sec. 2 potential
   V_M = q1 q2 / (4 pi eps0 sqrt(r^2 + a_c^2)) has one Coulomb constant for
   every ion; a_c = +inf is the exact harmonic bond; a finite a_c > 0 is used
   as given (and then fixes omega_c for the whole species). */
int or_add_species(or_ctx* c, int kind, double q1, double m1, double q2, double m2,
                   double weight, double omega_c, double a_c, double nu, double nu_per_omega,
                   double re_norm, int64_t capacity) {
  if (!c || c->nsp >= OR_MAX_SPECIES || capacity < 0) return -1;
  if (kind != OR_POINT && kind != OR_TWO_BODY) return -1;
  if (kind == OR_TWO_BODY) {
    if (!(omega_c > 0.0) || isnan(a_c) || a_c < 0.0) return -1;
    if (a_c == 0.0 && !(re_norm > 0.0)) return -1; /* a derived a_c must be positive */
  }
  or_species* s = &c->sp[c->nsp];
  memset(s, 0, sizeof(*s));
  s->kind = kind;
  s->q1 = q1;
  s->m1 = m1;
  s->q2 = q2;
  s->m2 = m2;
  s->weight = weight;
  s->omega_c = omega_c;
  s->a_c = a_c;
  s->nu = nu;
  s->nu_per_omega = nu_per_omega;
  s->ac_derived = kind == OR_TWO_BODY && a_c == 0.0;
  s->re_norm = re_norm;
  s->cap = capacity > 0 ? capacity : 1;
  s->cell = (int32_t*)calloc((size_t)s->cap * 3, sizeof(int32_t));
  s->off = (double*)calloc((size_t)s->cap * 3, sizeof(double));
  s->u1 = (double*)calloc((size_t)s->cap * 3, sizeof(double));
  if (kind == OR_TWO_BODY) {
    s->delta = (double*)calloc((size_t)s->cap * 3, sizeof(double));
    s->u2 = (double*)calloc((size_t)s->cap * 3, sizeof(double));
  }
  return c->nsp++;
}

/* Multi-shell ion (the extension the paper's summary names: the bound
   electrons split into several components): a nucleus (q0, m0) and nshell
   clouds, cloud k with charge qk[k], mass mk[k], bound to the nucleus alone
   by the softened bond of Sec. 2 with restoring frequency wk[k] and
   softening length ak[k] (0: derived from wk[k] with the Coulomb constant
   re_norm, as for a two-body ion; +inf: harmonic).  Each bond's reduced
   mass is that of its own pair, m0 mk / (m0 + mk), so one shell is exactly
   a two-body ion. */
int or_add_multishell(or_ctx* c, double q0, double m0, int nshell, const double* qk,
                      const double* mk, const double* wk, const double* ak, double weight,
                      double nu, double re_norm, int64_t capacity) {
  if (!c || c->nsp >= OR_MAX_SPECIES || capacity < 0) return -1;
  if (nshell < 1 || nshell > OR_MAX_SHELL || !qk || !mk || !wk || !ak) return -1;
  if (!(m0 > 0.0) || q0 == 0.0) return -1;
  for (int k = 0; k < nshell; k++) {
    if (!(mk[k] > 0.0) || qk[k] == 0.0 || !(wk[k] > 0.0) || isnan(ak[k]) || ak[k] < 0.0)
      return -1;
    if (ak[k] == 0.0 && !(re_norm > 0.0)) return -1;
  }
  or_species* s = &c->sp[c->nsp];
  memset(s, 0, sizeof(*s));
  s->kind = OR_MULTI_SHELL;
  s->q1 = q0;
  s->m1 = m0;
  s->nshell = nshell;
  for (int k = 0; k < nshell; k++) {
    s->qk[k] = qk[k];
    s->mk[k] = mk[k];
    s->wk[k] = wk[k];
    s->ak[k] = ak[k] == 0.0 ? or_ac_from_omega(q0, m0, qk[k], mk[k], wk[k], re_norm) : ak[k];
  }
  s->weight = weight;
  s->nu = nu;
  s->re_norm = re_norm;
  s->cap = capacity > 0 ? capacity : 1;
  s->cell = (int32_t*)calloc((size_t)s->cap * 3, sizeof(int32_t));
  s->off = (double*)calloc((size_t)s->cap * 3, sizeof(double));
  s->u1 = (double*)calloc((size_t)s->cap * 3, sizeof(double));
  s->delta = (double*)calloc((size_t)s->cap * 3 * nshell, sizeof(double));
  s->u2 = (double*)calloc((size_t)s->cap * 3 * nshell, sizeof(double));
  return c->nsp++;
}

/* Sec. 2 initial condition: p1 + p2 = p_c and q1 v1 + q2 v2 = 0, with
   p_i = m_i u_i and v_i = u_i / gamma_i.  Both velocities are parallel to
   u_c; v1 = alpha v2 with alpha = -q2/q1.  The speed s of body 2 solves
   m1 alpha s / sqrt(1 - alpha^2 s^2) + m2 s / sqrt(1 - s^2) = m_c |u_c|,
   which is increasing in s, so it is found by bisection. */
void or_split_momentum(double q1, double m1, double q2, double m2, const double* uc,
                       double* u1, double* u2) {
  double mc = m1 + m2;
  double norm = sqrt(uc[0] * uc[0] + uc[1] * uc[1] + uc[2] * uc[2]);
  if (norm == 0.0) {
    for (int a = 0; a < 3; a++) u1[a] = u2[a] = 0.0;
    return;
  }
  if (q1 + q2 == 0.0) { /* equal velocities: u1 = u2 = u_c */
    for (int a = 0; a < 3; a++) u1[a] = u2[a] = uc[a];
    return;
  }
  double alpha = -q2 / q1;
  double smax = 1.0;
  if (fabs(alpha) > 1.0) smax = 1.0 / fabs(alpha);
  double lo = 0.0, hi = smax, target = mc * norm;
  for (int it = 0; it < 200; it++) {
    double s = 0.5 * (lo + hi);
    double f = m1 * alpha * s / sqrt(1.0 - alpha * alpha * s * s) + m2 * s / sqrt(1.0 - s * s);
    if (f < target)
      lo = s;
    else
      hi = s;
  }
  double s = 0.5 * (lo + hi);
  double g2 = 1.0 / sqrt(1.0 - s * s);
  double g1 = 1.0 / sqrt(1.0 - alpha * alpha * s * s);
  for (int a = 0; a < 3; a++) {
    double e = uc[a] / norm;
    u2[a] = g2 * s * e;
    u1[a] = g1 * alpha * s * e;
  }
}

/* Physical position -> (cell, offset): xi = x / dx, cell = floor(xi), offset = xi - cell. */
static void to_cell(double x, double dx, int32_t* cell, double* off) {
  double xi = x / dx;
  double f = floor(xi);
  *cell = (int32_t)f;
  *off = xi - f;
}

int or_load_particles(or_ctx* c, int sid, int64_t n, const double* x, const double* delta,
                      const double* u1, const double* u2, const double* omega_c,
                      const double* weight) {
  if (!c || sid < 0 || sid >= c->nsp || n < 0 || (n > 0 && (!x || !u1))) return -1;
  or_species* s = &c->sp[sid];
  if (s->n + n > s->cap) return -2;
  if (s->kind == OR_MULTI_SHELL && omega_c) return -1; /* bond frequencies are per shell */
  if (omega_c && s->kind == OR_TWO_BODY) {
    /* a fixed finite a_c together with omega_c fixes the Coulomb constant,
       so the ions of such a species share one omega_c */
    if (!s->ac_derived && !isinf(s->a_c)) return -1;
    for (int64_t p = 0; p < n; p++)
      if (!(omega_c[p] > 0.0)) return -1;
  }
  if (omega_c && !s->wc) {
    if (s->n > 0) return -1;
    s->wc = (double*)calloc((size_t)s->cap, sizeof(double));
  }
  if (weight && !s->w) {
    if (s->n > 0) return -1;
    s->w = (double*)calloc((size_t)s->cap, sizeof(double));
  }
  for (int64_t p = 0; p < n; p++) {
    int64_t q = s->n + p;
    for (int d = 0; d < 3; d++) {
      if (d < c->nd) {
        to_cell(x[p * c->nd + d], c->g.dx[d], &s->cell[3 * q + d], &s->off[3 * q + d]);
        int32_t cl = s->cell[3 * q + d];
        if (cl < 0 || cl >= c->nn[d]) return -3;
        if (!periodic(c, d)) {
          double xi = (double)cl + s->off[3 * q + d];
          if (xi < (double)c->g.pad || xi > (double)(c->nn[d] - c->g.pad)) return -3;
        }
      } else {
        s->cell[3 * q + d] = 0;
        s->off[3 * q + d] = 0.0;
      }
    }
    if (s->kind == OR_MULTI_SHELL) {
      /* x is the centre of mass; body positions r0 = R + sum_k (m_k/M) d_k,
         r_k = r0 - d_k; every body between the walls.  u2 == NULL: every
         cloud moves with the nucleus. */
      const int K = s->nshell;
      double M = s->m1;
      for (int k = 0; k < K; k++) M += s->mk[k];
      for (int a = 0; a < 3 * K; a++) s->delta[3 * K * q + a] = delta ? delta[3 * K * p + a] : 0.0;
      for (int d = 0; d < c->nd; d++) {
        if (periodic(c, d)) continue;
        double X0 = (double)s->cell[3 * q + d] + s->off[3 * q + d];
        for (int k = 0; k < K; k++) X0 += (s->mk[k] / M) * s->delta[3 * K * q + 3 * k + d] / c->g.dx[d];
        double lo = (double)c->g.pad, hi = (double)(c->nn[d] - c->g.pad);
        if (!(X0 >= lo && X0 <= hi)) return -3;
        for (int k = 0; k < K; k++) {
          double Xk = X0 - s->delta[3 * K * q + 3 * k + d] / c->g.dx[d];
          if (!(Xk >= lo && Xk <= hi)) return -3;
        }
      }
      for (int a = 0; a < 3; a++) s->u1[3 * q + a] = u1[3 * p + a];
      for (int k = 0; k < K; k++)
        for (int a = 0; a < 3; a++)
          s->u2[3 * K * q + 3 * k + a] = u2 ? u2[3 * K * p + 3 * k + a] : u1[3 * p + a];
    } else if (s->kind == OR_TWO_BODY) {
      for (int a = 0; a < 3; a++) s->delta[3 * q + a] = delta ? delta[3 * p + a] : 0.0;
      /* along walled axes both bodies lie between the walls */
      double mc = s->m1 + s->m2;
      for (int d = 0; d < c->nd; d++) {
        if (periodic(c, d)) continue;
        double X = (double)s->cell[3 * q + d] + s->off[3 * q + d];
        double sd = s->delta[3 * q + d] / c->g.dx[d];
        double X1 = X + (s->m2 / mc) * sd, X2 = X - (s->m1 / mc) * sd;
        double lo = (double)c->g.pad, hi = (double)(c->nn[d] - c->g.pad);
        if (!(X1 >= lo && X1 <= hi && X2 >= lo && X2 <= hi)) return -3;
      }
      if (u2) {
        for (int a = 0; a < 3; a++) {
          s->u1[3 * q + a] = u1[3 * p + a];
          s->u2[3 * q + a] = u2[3 * p + a];
        }
      } else {
        or_split_momentum(s->q1, s->m1, s->q2, s->m2, &u1[3 * p], &s->u1[3 * q], &s->u2[3 * q]);
      }
    } else {
      for (int a = 0; a < 3; a++) s->u1[3 * q + a] = u1[3 * p + a];
    }
    if (s->wc) s->wc[q] = omega_c ? omega_c[p] : s->omega_c;
    if (s->w) s->w[q] = weight ? weight[p] : s->weight;
  }
  s->n += n;
  return 0;
}

int64_t or_count(or_ctx* c, int sid) {
  if (!c || sid < 0 || sid >= c->nsp) return -1;
  return c->sp[sid].n;
}

int or_load_fields(or_ctx* c, const double* E, const double* B) {
  if (!c) return -1;
  for (int64_t k = 0; k < c->nn[2]; k++)
    for (int64_t j = 0; j < c->nn[1]; j++)
      for (int64_t i = 0; i < c->nn[0]; i++) {
        int64_t f = fidx(c, i, j, k), q = cidx(c, i, j, k);
        for (int a = 0; a < 3; a++) {
          c->E[a][f] = E ? E[a * c->ncell + q] : 0.0;
          c->B[a][f] = B ? B[a * c->ncell + q] : 0.0;
        }
      }
  return 0;
}

int or_read_fields(or_ctx* c, double* E, double* B, double* J) {
  if (!c) return -1;
  for (int64_t k = 0; k < c->nn[2]; k++)
    for (int64_t j = 0; j < c->nn[1]; j++)
      for (int64_t i = 0; i < c->nn[0]; i++) {
        int64_t f = fidx(c, i, j, k), q = cidx(c, i, j, k);
        for (int a = 0; a < 3; a++) {
          if (E) E[a * c->ncell + q] = c->E[a][f];
          if (B) B[a * c->ncell + q] = c->B[a][f];
          if (J) J[a * c->ncell + q] = c->J[a][f];
        }
      }
  return 0;
}

int or_read_particles(or_ctx* c, int sid, int32_t* cell, double* off, double* delta,
                      double* u1, double* u2) {
  if (!c || sid < 0 || sid >= c->nsp) return -1;
  or_species* s = &c->sp[sid];
  size_t m = (size_t)s->n * 3;
  size_t mk = m * (size_t)(s->kind == OR_MULTI_SHELL ? s->nshell : 1);
  if (cell) memcpy(cell, s->cell, m * sizeof(int32_t));
  if (off) memcpy(off, s->off, m * sizeof(double));
  if (delta && s->delta) memcpy(delta, s->delta, mk * sizeof(double));
  if (u1) memcpy(u1, s->u1, m * sizeof(double));
  if (u2 && s->u2) memcpy(u2, s->u2, mk * sizeof(double));
  return 0;
}

/* ----------------------------------------------------------------- gather */

/* Field components and their Yee stagger: component a sits half a cell off
   the node along the dimensions with stag = 1.
   E_x (1/2,0,0)  E_y (0,1/2,0)  E_z (0,0,1/2)
   B_x (0,1/2,1/2) B_y (1/2,0,1/2) B_z (1/2,1/2,0) */
static const int STAG_E[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
static const int STAG_B[3][3] = {{0, 1, 1}, {1, 0, 1}, {1, 1, 0}};

/* Interpolate one field component at a position given relative to a cell:
   sum over nodes of S(xi - node) * F(node), with S the quadratic B-spline
   and the node positions shifted by the component's stagger. */
static double interp(or_ctx* c, const double* F, const int stag[3], const int32_t cell[3],
                     const double xi[3]) {
  double w[3][NW];
  int lo[3], hi[3];
  for (int d = 0; d < 3; d++) {
    if (resolved(c, d)) {
      lo[d] = 0;
      hi[d] = NW;
      for (int r = 0; r < NW; r++) w[d][r] = b2(xi[d] - (double)(r + RLO) - 0.5 * stag[d]);
    } else {
      lo[d] = 0;
      hi[d] = 1;
      w[d][0] = 1.0;
    }
  }
  double sum = 0.0;
  for (int t = lo[2]; t < hi[2]; t++)
    for (int s = lo[1]; s < hi[1]; s++)
      for (int r = lo[0]; r < hi[0]; r++) {
        double wt = w[0][r] * w[1][s] * w[2][t];
        if (wt == 0.0) continue;
        int64_t i = resolved(c, 0) ? (int64_t)cell[0] + r + RLO : 0;
        int64_t j = resolved(c, 1) ? (int64_t)cell[1] + s + RLO : 0;
        int64_t k = resolved(c, 2) ? (int64_t)cell[2] + t + RLO : 0;
        if (!wrap(c, 0, &i) || !wrap(c, 1, &j) || !wrap(c, 2, &k)) {
          c->err |= OR_ERR_RANGE;
          continue;
        }
        sum += wt * F[fidx(c, i, j, k)];
      }
  return sum;
}

static void gather(or_ctx* c, const int32_t cell[3], const double xi[3], double E[3], double B[3]) {
  for (int a = 0; a < 3; a++) {
    E[a] = interp(c, c->E[a], STAG_E[a], cell, xi);
    B[a] = interp(c, c->B[a], STAG_B[a], cell, xi);
  }
}

int or_gather(or_ctx* c, const int32_t* cell, const double* off, double* E, double* B) {
  if (!c) return -1;
  int32_t cl[3] = {0, 0, 0};
  double xi[3] = {0, 0, 0};
  for (int d = 0; d < c->nd; d++) {
    cl[d] = cell[d];
    xi[d] = off[d];
  }
  gather(c, cl, xi, E, B);
  return 0;
}

/* ---------------------------------------------------------------- deposit */

static void jadd(or_ctx* c, int a, int64_t i, int64_t j, int64_t k, double v) {
  if (v == 0.0) return;
  if (!wrap(c, 0, &i) || !wrap(c, 1, &j) || !wrap(c, 2, &k)) {
    c->err |= OR_ERR_RANGE;
    return;
  }
  c->J[a][fidx(c, i, j, k)] += v;
}

/* Esirkepov (2001) charge-conserving current of one body of charge Q
   (= real charge x weight) moving from x0 to x1 (cell units, relative to
   `cell`; x0 in [0, 1), so the window -2 .. +3 holds both shapes).  v is
   the body velocity, used for the components along unresolved dimensions,
   which carry the time-averaged shape.  Along its own axis a component is
   the running sum of the shape change; at the window's last node that sum
   runs over the whole of both shapes and is zero (the body's charge is
   conserved), so the running sums stop one node short of it. */
static void deposit(or_ctx* c, const int32_t cell[3], const double x0[3], const double x1[3],
                    double Q, const double v[3]) {
  const or_config* g = &c->g;
  int nd = c->nd;
  double S0[3][NW], DS[3][NW];
  double dV = 1.0;
  for (int d = 0; d < nd; d++) {
    dV *= g->dx[d];
    for (int r = 0; r < NW; r++) {
      double a = b2(x0[d] - (double)(r + RLO));
      double b = b2(x1[d] - (double)(r + RLO));
      S0[d][r] = a;
      DS[d][r] = b - a;
    }
  }
  int64_t ci = cell[0], cj = nd > 1 ? cell[1] : 0, ck = nd > 2 ? cell[2] : 0;
  if (nd == 1) {
    double fx = -Q * g->dx[0] / (g->dt * dV);
    double acc = 0.0;
    for (int r = 0; r < NW; r++) {
      acc += DS[0][r];
      if (r < NW - 1) jadd(c, 0, ci + r + RLO, 0, 0, fx * acc);
      double sh = S0[0][r] + 0.5 * DS[0][r];
      jadd(c, 1, ci + r + RLO, 0, 0, Q * v[1] / dV * sh);
      jadd(c, 2, ci + r + RLO, 0, 0, Q * v[2] / dV * sh);
    }
  } else if (nd == 2) {
    double fx = -Q * g->dx[0] / (g->dt * dV);
    double fy = -Q * g->dx[1] / (g->dt * dV);
    for (int s = 0; s < NW; s++) {
      double acc = 0.0;
      for (int r = 0; r < NW - 1; r++) {
        acc += DS[0][r] * (S0[1][s] + 0.5 * DS[1][s]);
        jadd(c, 0, ci + r + RLO, cj + s + RLO, 0, fx * acc);
      }
    }
    for (int r = 0; r < NW; r++) {
      double acc = 0.0;
      for (int s = 0; s < NW - 1; s++) {
        acc += DS[1][s] * (S0[0][r] + 0.5 * DS[0][r]);
        jadd(c, 1, ci + r + RLO, cj + s + RLO, 0, fy * acc);
      }
    }
    for (int s = 0; s < NW; s++)
      for (int r = 0; r < NW; r++) {
        double wz = S0[0][r] * S0[1][s] + 0.5 * DS[0][r] * S0[1][s] + 0.5 * S0[0][r] * DS[1][s] +
                    DS[0][r] * DS[1][s] / 3.0;
        jadd(c, 2, ci + r + RLO, cj + s + RLO, 0, Q * v[2] / dV * wz);
      }
  } else {
    double f[3];
    for (int d = 0; d < 3; d++) f[d] = -Q * g->dx[d] / (g->dt * dV);
    /* W_x, summed along x */
    for (int t = 0; t < NW; t++)
      for (int s = 0; s < NW; s++) {
        double acc = 0.0;
        for (int r = 0; r < NW - 1; r++) {
          acc += DS[0][r] * (S0[1][s] * S0[2][t] + 0.5 * DS[1][s] * S0[2][t] +
                             0.5 * S0[1][s] * DS[2][t] + DS[1][s] * DS[2][t] / 3.0);
          jadd(c, 0, ci + r + RLO, cj + s + RLO, ck + t + RLO, f[0] * acc);
        }
      }
    /* W_y, summed along y */
    for (int t = 0; t < NW; t++)
      for (int r = 0; r < NW; r++) {
        double acc = 0.0;
        for (int s = 0; s < NW - 1; s++) {
          acc += DS[1][s] * (S0[0][r] * S0[2][t] + 0.5 * DS[0][r] * S0[2][t] +
                             0.5 * S0[0][r] * DS[2][t] + DS[0][r] * DS[2][t] / 3.0);
          jadd(c, 1, ci + r + RLO, cj + s + RLO, ck + t + RLO, f[1] * acc);
        }
      }
    /* W_z, summed along z */
    for (int s = 0; s < NW; s++)
      for (int r = 0; r < NW; r++) {
        double acc = 0.0;
        for (int t = 0; t < NW - 1; t++) {
          acc += DS[2][t] * (S0[0][r] * S0[1][s] + 0.5 * DS[0][r] * S0[1][s] +
                             0.5 * S0[0][r] * DS[1][s] + DS[0][r] * DS[1][s] / 3.0);
          jadd(c, 2, ci + r + RLO, cj + s + RLO, ck + t + RLO, f[2] * acc);
        }
      }
  }
}

/* ------------------------------------------------------------------- push */

/* Sec. 2: each body of a two-body ion has its own position.  A body at x
   (cell units, relative to the centre's cell `cell`) is gathered and
   deposited in the frame of the cell that holds it: cell + floor(x), offset
   x - floor(x) (an exact subtraction), so its windows follow it however far
   it is from the centre of mass. */
static void body_frame(const or_ctx* c, const int32_t cell[3], const double x[3],
                       int32_t bc[3], double bx[3]) {
  for (int d = 0; d < 3; d++) {
    if (resolved(c, d)) {
      double k = floor(x[d]);
      bc[d] = cell[d] + (int32_t)k;
      bx[d] = x[d] - k;
    } else {
      bc[d] = 0;
      bx[d] = 0.0;
    }
  }
}

/* Along an axis with walls a body stays between the walls `pad` cells
   inside the faces (they mirror every body that reaches them), where every
   node its shape reaches is interior.  x is relative to `cell`. */
static int body_in_range(const or_ctx* c, const int32_t cell[3], const double x[3]) {
  for (int d = 0; d < c->nd; d++) {
    if (periodic(c, d)) continue;
    if (!(x[d] >= (double)(c->g.pad - cell[d]) && x[d] <= (double)(c->nn[d] - c->g.pad - cell[d])))
      return 0;
  }
  return 1;
}

/* Boris rotation and second half kick of one body (Sec. 2):
   t = (q dt / 2m) B / gamma^-, s = 2t / (1 + t^2),
   u+ = u- + (u- + u- x t) x s,  u^{new} = u+ + (q dt / 2m) E. */
static void boris_finish(const double um[3], double a, const double E[3], const double B[3],
                         double out[3]) {
  double gm = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
  double t[3], s[3], w[3], up[3];
  for (int k = 0; k < 3; k++) t[k] = a * B[k] / gm;
  double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
  for (int k = 0; k < 3; k++) s[k] = 2.0 * t[k] / (1.0 + t2);
  w[0] = um[0] + (um[1] * t[2] - um[2] * t[1]);
  w[1] = um[1] + (um[2] * t[0] - um[0] * t[2]);
  w[2] = um[2] + (um[0] * t[1] - um[1] * t[0]);
  up[0] = um[0] + (w[1] * s[2] - w[2] * s[1]);
  up[1] = um[1] + (w[2] * s[0] - w[0] * s[2]);
  up[2] = um[2] + (w[0] * s[1] - w[1] * s[0]);
  for (int k = 0; k < 3; k++) out[k] = up[k] + a * E[k];
}

/* Reflecting particle walls, `pad` cells inside each non-periodic face, for
   a point particle (the bodies of a two-body ion reflect one by one, see
   push_two_body).  off is the new offset relative to the old cell (not yet
   wrapped).  Returns 1 when the particle was mirrored. */
static int reflect(or_ctx* c, int d, int32_t cell, double* off) {
  if (periodic(c, d)) return 0;
  int64_t wl = c->g.pad, wr = c->nn[d] - c->g.pad;
  if (cell == wl && *off < 0.0) {
    *off = -*off;
    return 1;
  }
  if (cell == wr - 1 && *off > 1.0) {
    *off = 2.0 - *off;
    return 1;
  }
  if (cell == wr && *off > 0.0) {
    *off = -*off;
    return 1;
  }
  return 0;
}

/* Integer cell-crossing rule: offset >= 1 moves one cell up, offset < 0
   one cell down (at most one crossing per step under the CFL limit). */
static void cross(or_ctx* c, int d, int32_t* cell, double* off) {
  if (*off >= 1.0) {
    *cell += 1;
    *off -= 1.0;
  } else if (*off < 0.0) {
    *cell -= 1;
    *off += 1.0;
  }
  if (periodic(c, d)) {
    if (*cell >= c->nn[d]) *cell -= (int32_t)c->nn[d];
    if (*cell < 0) *cell += (int32_t)c->nn[d];
  }
}

static void push_two_body(or_ctx* c, or_species* s, int64_t p) {
  const or_config* g = &c->g;
  int nd = c->nd;
  double q1 = s->q1, m1 = s->m1, q2 = s->q2, m2 = s->m2;
  double mc = m1 + m2, f1 = m2 / mc, f2 = m1 / mc, mr = m1 * m2 / mc;
  double wc = s->wc ? s->wc[p] : s->omega_c;
  double nu = s->nu + s->nu_per_omega * wc;
  double W = s->w ? s->w[p] : s->weight;
  /* the ion's own softening length (Sec. 3.1 with its own omega_c) */
  double ac = s->ac_derived ? or_ac_from_omega(q1, m1, q2, m2, wc, s->re_norm) : s->a_c;
  int32_t* cell = &s->cell[3 * p];
  double* off = &s->off[3 * p];
  double* dl = &s->delta[3 * p];
  double* u1 = &s->u1[3 * p];
  double* u2 = &s->u2[3 * p];

  /* body positions r1 = r_c + (m2/m_c) r, r2 = r_c - (m1/m_c) r (Sec. 3.1),
     relative to the centre's cell, and each body's own cell frame */
  double x1[3] = {0, 0, 0}, x2[3] = {0, 0, 0};
  for (int d = 0; d < nd; d++) {
    x1[d] = off[d] + f1 * dl[d] / g->dx[d];
    x2[d] = off[d] - f2 * dl[d] / g->dx[d];
  }
  int32_t c1[3], c2[3];
  double b1[3], b2_[3];
  body_frame(c, cell, x1, c1, b1);
  body_frame(c, cell, x2, c2, b2_);
  double E1[3], B1[3], E2[3], B2[3];
  gather(c, c1, b1, E1, B1);
  gather(c, c2, b2_, E2, B2);

  /* internal softened-Coulomb force on the nucleus,
     F = q1 q2 r / (4 pi eps0 (r^2 + a_c^2)^{3/2}) = -m_r w_c^2 r (1 + r^2/a_c^2)^{-3/2},
     +F on body 1 and -F on body 2, entering the push as extra E. */
  double r2 = dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2];
  double soft = isinf(ac) ? 1.0 : pow(1.0 + r2 / (ac * ac), -1.5);
  double kf = -mr * wc * wc * soft;
  for (int a = 0; a < 3; a++) {
    double F = kf * dl[a];
    E1[a] += F / q1;
    E2[a] -= F / q2;
  }
  double h = 0.5 * g->dt;
  double a1 = h * q1 / m1, a2 = h * q2 / m2;
  double um1[3], um2[3];
  for (int a = 0; a < 3; a++) {
    um1[a] = u1[a] + a1 * E1[a];
    um2[a] = u2[a] + a2 * E2[a];
  }
  if (nu > 0.0) {
    /* friction on the relative momentum, total momentum m1 u1 + m2 u2 kept */
    double D = (1.0 - nu * h) / (1.0 + nu * h);
    for (int a = 0; a < 3; a++) {
      double V = (m1 * um1[a] + m2 * um2[a]) / mc;
      double w = (um1[a] - um2[a]) * D;
      um1[a] = V + f1 * w;
      um2[a] = V - f2 * w;
    }
  }
  double n1[3], n2[3];
  boris_finish(um1, a1, E1, B1, n1);
  boris_finish(um2, a2, E2, B2, n2);
  double g1 = sqrt(1.0 + n1[0] * n1[0] + n1[1] * n1[1] + n1[2] * n1[2]);
  double g2 = sqrt(1.0 + n2[0] * n2[0] + n2[1] * n2[1] + n2[2] * n2[2]);
  double v1[3], v2[3];
  for (int a = 0; a < 3; a++) {
    v1[a] = n1[a] / g1;
    v2[a] = n2[a] / g2;
    u1[a] = n1[a];
    u2[a] = n2[a];
  }

  /* move: R += dt (m1 v1 + m2 v2)/m_c, delta += dt (v1 - v2) */
  double offn[3] = {0, 0, 0};
  for (int a = 0; a < 3; a++) dl[a] = dl[a] + g->dt * (v1[a] - v2[a]);
  for (int d = 0; d < nd; d++) offn[d] = off[d] + g->dt * (m1 * v1[d] + m2 * v2[d]) / mc / g->dx[d];
  /* Reflecting walls act on each body, a particle with its own position
     (Sec. 2): a body past a wall is mirrored back (moved by D cells) and its
     momentum component reversed; R moves by (m_i/m_c) D and delta by +-D dx. */
  for (int d = 0; d < nd; d++) {
    if (periodic(c, d)) continue;
    double lo = (double)(g->pad - cell[d]), hi = (double)(c->nn[d] - g->pad - cell[d]);
    double s = dl[d] / g->dx[d];
    double y[2] = {offn[d] + f1 * s, offn[d] - f2 * s}, D[2] = {0.0, 0.0};
    for (int b = 0; b < 2; b++) {
      if (y[b] < lo) D[b] = 2.0 * (lo - y[b]);
      else if (y[b] > hi) D[b] = 2.0 * (hi - y[b]);
    }
    if (D[0] != 0.0) u1[d] = -u1[d];
    if (D[1] != 0.0) u2[d] = -u2[d];
    if (D[0] != 0.0 || D[1] != 0.0) {
      offn[d] += f2 * D[0] + f1 * D[1];
      dl[d] += (D[0] - D[1]) * g->dx[d];
    }
  }
  /* new body positions, relative to the centre's old cell and in each
     body's old frame */
  double y1[3] = {0, 0, 0}, y2[3] = {0, 0, 0};
  for (int d = 0; d < nd; d++) {
    y1[d] = offn[d] + f1 * dl[d] / g->dx[d];
    y2[d] = offn[d] - f2 * dl[d] / g->dx[d];
  }
  if (!(g->flags & OR_NO_DEPOSIT)) {
    double z1[3] = {0, 0, 0}, z2[3] = {0, 0, 0};
    for (int d = 0; d < nd; d++) {
      z1[d] = y1[d] - (double)(c1[d] - cell[d]);
      z2[d] = y2[d] - (double)(c2[d] - cell[d]);
    }
    deposit(c, c1, b1, z1, q1 * W, v1);
    deposit(c, c2, b2_, z2, q2 * W, v2);
  }
  if (!body_in_range(c, cell, y1) || !body_in_range(c, cell, y2)) c->err |= OR_ERR_RANGE;
  for (int d = 0; d < nd; d++) {
    cross(c, d, &cell[d], &offn[d]);
    off[d] = offn[d];
  }
  for (int a = 0; a < 3; a++)
    if (!isfinite(u1[a]) || !isfinite(u2[a]) || !isfinite(dl[a])) c->err |= OR_ERR_NAN;
}

/* One step of a multi-shell ion, the two-body step of Sec. 2 with one
   bond per shell: every body is gathered at its own position, each bond
   adds +F_k / q0 to the nucleus' field and -F_k / q_k to cloud k's, each
   body is Boris-pushed, the centre of mass moves with the mass-weighted
   velocities and d_k = r0 - r_k with v0 - v_k, the walls mirror each body,
   and each body deposits its own current.  The damping nu acts on each
   nucleus-cloud pair in turn as on a two-body ion (pair momentum kept). */
static void push_multishell(or_ctx* c, or_species* s, int64_t p) {
  const or_config* g = &c->g;
  const int nd = c->nd, K = s->nshell, nb = K + 1;
  double W = s->w ? s->w[p] : s->weight;
  double q[OR_MAX_SHELL + 1], m[OR_MAX_SHELL + 1];
  q[0] = s->q1;
  m[0] = s->m1;
  double M = s->m1;
  for (int k = 0; k < K; k++) {
    q[k + 1] = s->qk[k];
    m[k + 1] = s->mk[k];
    M += s->mk[k];
  }
  int32_t* cell = &s->cell[3 * p];
  double* off = &s->off[3 * p];
  double* dl = &s->delta[3 * K * p]; /* shell k at dl + 3k */
  double* u[OR_MAX_SHELL + 1];
  u[0] = &s->u1[3 * p];
  for (int k = 0; k < K; k++) u[k + 1] = &s->u2[3 * K * p + 3 * k];

  /* body positions (cell units, relative to the centre's cell) and frames */
  double x[OR_MAX_SHELL + 1][3];
  memset(x, 0, sizeof(x));
  for (int d = 0; d < nd; d++) {
    double r0 = off[d];
    for (int k = 0; k < K; k++) r0 += (m[k + 1] / M) * dl[3 * k + d] / g->dx[d];
    x[0][d] = r0;
    for (int k = 0; k < K; k++) x[k + 1][d] = r0 - dl[3 * k + d] / g->dx[d];
  }
  int32_t bc[OR_MAX_SHELL + 1][3];
  double bx[OR_MAX_SHELL + 1][3], E[OR_MAX_SHELL + 1][3], B[OR_MAX_SHELL + 1][3];
  for (int b = 0; b < nb; b++) {
    body_frame(c, cell, x[b], bc[b], bx[b]);
    gather(c, bc[b], bx[b], E[b], B[b]);
  }
  /* the bonds, as extra fields */
  for (int k = 0; k < K; k++) {
    const double* r = &dl[3 * k];
    double mr = m[0] * m[k + 1] / (m[0] + m[k + 1]);
    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double ak = s->ak[k];
    double soft = isinf(ak) ? 1.0 : pow(1.0 + r2 / (ak * ak), -1.5);
    double kf = -mr * s->wk[k] * s->wk[k] * soft;
    for (int a = 0; a < 3; a++) {
      double F = kf * r[a];
      E[0][a] += F / q[0];
      E[k + 1][a] -= F / q[k + 1];
    }
  }
  double h = 0.5 * g->dt;
  double ab[OR_MAX_SHELL + 1], um[OR_MAX_SHELL + 1][3];
  for (int b = 0; b < nb; b++) {
    ab[b] = h * q[b] / m[b];
    for (int a = 0; a < 3; a++) um[b][a] = u[b][a] + ab[b] * E[b][a];
  }
  if (s->nu > 0.0) {
    double D = (1.0 - s->nu * h) / (1.0 + s->nu * h);
    for (int k = 0; k < K; k++) {
      double mp = m[0] + m[k + 1];
      for (int a = 0; a < 3; a++) {
        double V = (m[0] * um[0][a] + m[k + 1] * um[k + 1][a]) / mp;
        double w = (um[0][a] - um[k + 1][a]) * D;
        um[0][a] = V + (m[k + 1] / mp) * w;
        um[k + 1][a] = V - (m[0] / mp) * w;
      }
    }
  }
  double v[OR_MAX_SHELL + 1][3];
  for (int b = 0; b < nb; b++) {
    double nw[3];
    boris_finish(um[b], ab[b], E[b], B[b], nw);
    double gm = sqrt(1.0 + nw[0] * nw[0] + nw[1] * nw[1] + nw[2] * nw[2]);
    for (int a = 0; a < 3; a++) {
      u[b][a] = nw[a];
      v[b][a] = nw[a] / gm;
    }
  }
  /* move */
  double offn[3] = {0, 0, 0};
  for (int k = 0; k < K; k++)
    for (int a = 0; a < 3; a++) dl[3 * k + a] += g->dt * (v[0][a] - v[k + 1][a]);
  for (int d = 0; d < nd; d++) {
    double P = 0.0;
    for (int b = 0; b < nb; b++) P += m[b] * v[b][d];
    offn[d] = off[d] + g->dt * P / M / g->dx[d];
  }
  /* walls: a body past a wall is mirrored (moved by D cells) and its
     momentum component reversed; R moves by (m_b/M) D; the nucleus' move
     adds D dx to every d_k, cloud k's subtracts it from d_k */
  for (int d = 0; d < nd; d++) {
    if (periodic(c, d)) continue;
    double lo = (double)(g->pad - cell[d]), hi = (double)(c->nn[d] - g->pad - cell[d]);
    double y[OR_MAX_SHELL + 1], Dm[OR_MAX_SHELL + 1];
    double y0 = offn[d];
    for (int k = 0; k < K; k++) y0 += (m[k + 1] / M) * dl[3 * k + d] / g->dx[d];
    y[0] = y0;
    for (int k = 0; k < K; k++) y[k + 1] = y0 - dl[3 * k + d] / g->dx[d];
    for (int b = 0; b < nb; b++) {
      Dm[b] = 0.0;
      if (y[b] < lo) Dm[b] = 2.0 * (lo - y[b]);
      else if (y[b] > hi) Dm[b] = 2.0 * (hi - y[b]);
      if (Dm[b] != 0.0) {
        u[b][d] = -u[b][d];
        offn[d] += (m[b] / M) * Dm[b];
      }
    }
    for (int k = 0; k < K; k++) dl[3 * k + d] += (Dm[0] - Dm[k + 1]) * g->dx[d];
  }
  /* new body positions, relative to the centre's old cell */
  double yb[OR_MAX_SHELL + 1][3];
  memset(yb, 0, sizeof(yb));
  for (int d = 0; d < nd; d++) {
    double r0 = offn[d];
    for (int k = 0; k < K; k++) r0 += (m[k + 1] / M) * dl[3 * k + d] / g->dx[d];
    yb[0][d] = r0;
    for (int k = 0; k < K; k++) yb[k + 1][d] = r0 - dl[3 * k + d] / g->dx[d];
  }
  if (!(g->flags & OR_NO_DEPOSIT)) {
    for (int b = 0; b < nb; b++) {
      double z[3] = {0, 0, 0};
      for (int d = 0; d < nd; d++) z[d] = yb[b][d] - (double)(bc[b][d] - cell[d]);
      deposit(c, bc[b], bx[b], z, q[b] * W, v[b]);
    }
  }
  for (int b = 0; b < nb; b++)
    if (!body_in_range(c, cell, yb[b])) c->err |= OR_ERR_RANGE;
  for (int d = 0; d < nd; d++) {
    cross(c, d, &cell[d], &offn[d]);
    off[d] = offn[d];
  }
  for (int b = 0; b < nb; b++)
    for (int a = 0; a < 3; a++)
      if (!isfinite(u[b][a])) c->err |= OR_ERR_NAN;
  for (int a = 0; a < 3 * K; a++)
    if (!isfinite(dl[a])) c->err |= OR_ERR_NAN;
}

static void push_point(or_ctx* c, or_species* s, int64_t p) {
  const or_config* g = &c->g;
  int nd = c->nd;
  double q = s->q1, m = s->m1;
  double W = s->w ? s->w[p] : s->weight;
  int32_t* cell = &s->cell[3 * p];
  double* off = &s->off[3 * p];
  double* u = &s->u1[3 * p];
  double x0[3] = {0, 0, 0};
  for (int d = 0; d < nd; d++) x0[d] = off[d];
  double E[3], B[3];
  gather(c, cell, x0, E, B);
  double a = 0.5 * g->dt * q / m;
  double um[3], n[3];
  for (int k = 0; k < 3; k++) um[k] = u[k] + a * E[k];
  boris_finish(um, a, E, B, n);
  double gm = sqrt(1.0 + n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  double v[3];
  for (int k = 0; k < 3; k++) {
    v[k] = n[k] / gm;
    u[k] = n[k];
  }
  double x1[3] = {0, 0, 0};
  for (int d = 0; d < nd; d++) {
    x1[d] = off[d] + g->dt * v[d] / g->dx[d];
    if (reflect(c, d, cell[d], &x1[d])) u[d] = -u[d];
  }
  if (!(g->flags & OR_NO_DEPOSIT)) deposit(c, cell, x0, x1, q * W, v);
  for (int d = 0; d < nd; d++) {
    cross(c, d, &cell[d], &x1[d]);
    off[d] = x1[d];
  }
  for (int k = 0; k < 3; k++)
    if (!isfinite(u[k])) c->err |= OR_ERR_NAN;
}

/* ---------------------------------------------------------------- density */

static void add_rho(or_ctx* c, double* rho, const int32_t cell[3], const double x[3], double Q) {
  double w[3][NW];
  int hi[3];
  double dV = 1.0;
  for (int d = 0; d < 3; d++) {
    if (resolved(c, d)) {
      dV *= c->g.dx[d];
      hi[d] = NW;
      for (int r = 0; r < NW; r++) w[d][r] = b2(x[d] - (double)(r + RLO));
    } else {
      hi[d] = 1;
      w[d][0] = 1.0;
    }
  }
  for (int t = 0; t < hi[2]; t++)
    for (int s = 0; s < hi[1]; s++)
      for (int r = 0; r < hi[0]; r++) {
        double wt = w[0][r] * w[1][s] * w[2][t];
        if (wt == 0.0) continue;
        int64_t i = resolved(c, 0) ? (int64_t)cell[0] + r + RLO : 0;
        int64_t j = resolved(c, 1) ? (int64_t)cell[1] + s + RLO : 0;
        int64_t k = resolved(c, 2) ? (int64_t)cell[2] + t + RLO : 0;
        if (!wrap(c, 0, &i) || !wrap(c, 1, &j) || !wrap(c, 2, &k)) {
          c->err |= OR_ERR_RANGE;
          continue;
        }
        rho[cidx(c, i, j, k)] += Q * wt / dV;
      }
}

int or_rho(or_ctx* c, double* rho) {
  if (!c || !rho) return -1;
  memset(rho, 0, (size_t)c->ncell * sizeof(double));
  for (int si = 0; si < c->nsp; si++) {
    or_species* s = &c->sp[si];
    for (int64_t p = 0; p < s->n; p++) {
      double W = s->w ? s->w[p] : s->weight;
      const int32_t* cell = &s->cell[3 * p];
      const double* off = &s->off[3 * p];
      double x[3] = {0, 0, 0};
      if (s->kind == OR_MULTI_SHELL) {
        const int K = s->nshell;
        const double* dl = &s->delta[3 * K * p];
        double M = s->m1;
        for (int k = 0; k < K; k++) M += s->mk[k];
        double x0[3] = {0, 0, 0};
        for (int d = 0; d < c->nd; d++) {
          x0[d] = off[d];
          for (int k = 0; k < K; k++) x0[d] += (s->mk[k] / M) * dl[3 * k + d] / c->g.dx[d];
        }
        int32_t bc[3];
        double bx[3];
        body_frame(c, cell, x0, bc, bx);
        add_rho(c, rho, bc, bx, s->q1 * W);
        for (int k = 0; k < K; k++) {
          for (int d = 0; d < c->nd; d++) x[d] = x0[d] - dl[3 * k + d] / c->g.dx[d];
          body_frame(c, cell, x, bc, bx);
          add_rho(c, rho, bc, bx, s->qk[k] * W);
        }
      } else if (s->kind == OR_TWO_BODY) {
        double mc = s->m1 + s->m2, f1 = s->m2 / mc, f2 = s->m1 / mc;
        const double* dl = &s->delta[3 * p];
        int32_t bc[3];
        double bx[3];
        for (int d = 0; d < c->nd; d++) x[d] = off[d] + f1 * dl[d] / c->g.dx[d];
        body_frame(c, cell, x, bc, bx);
        add_rho(c, rho, bc, bx, s->q1 * W);
        for (int d = 0; d < c->nd; d++) x[d] = off[d] - f2 * dl[d] / c->g.dx[d];
        body_frame(c, cell, x, bc, bx);
        add_rho(c, rho, bc, bx, s->q2 * W);
      } else {
        for (int d = 0; d < c->nd; d++) x[d] = off[d];
        add_rho(c, rho, cell, x, s->q1 * W);
      }
    }
  }
  return 0;
}

/* ------------------------------------------------------------- field solve */

/* coordinates of a face-plane node: dim d fixed at p, (a, b) over the other dims */
static void face_ijk(int d, int64_t p, int64_t a, int64_t b, int64_t* i, int64_t* j, int64_t* k) {
  if (d == 0) {
    *i = p;
    *j = a;
    *k = b;
  } else if (d == 1) {
    *i = a;
    *j = p;
    *k = b;
  } else {
    *i = a;
    *j = b;
    *k = p;
  }
}
static void face_extent(const or_ctx* c, int d, int64_t* na, int64_t* nb) {
  if (d == 0) {
    *na = c->nn[1];
    *nb = c->nn[2];
  } else if (d == 1) {
    *na = c->nn[0];
    *nb = c->nn[2];
  } else {
    *na = c->nn[0];
    *nb = c->nn[1];
  }
}
/* the two field components tangential to a face normal to d */
static void tangential(int d, int* t0, int* t1) {
  *t0 = d == 0 ? 1 : 0;
  *t1 = d == 2 ? 1 : 2;
}

/* Cardinal cubic B-spline: the fourfold convolution of the unit box,
   supported on [0, 4], one cubic piece per unit interval (de Boor). */
static double cubic_bspline(double s) {
  if (s <= 0.0 || s >= 4.0) return 0.0;
  if (s < 1.0) return s * s * s / 6.0;
  if (s < 2.0) return (-3.0 * s * s * s + 12.0 * s * s - 12.0 * s + 4.0) / 6.0;
  if (s < 3.0) return (3.0 * s * s * s - 24.0 * s * s + 60.0 * s - 44.0) / 6.0;
  return (4.0 - s) * (4.0 - s) * (4.0 - s) / 6.0;
}

/* Temporal envelope of the laser: sin^2 over [0, t_env], or the sum of the
   n_env spline coefficients times their basis functions. */
static double envelope(const or_config* g, double tau) {
  if (g->n_env <= 0) {
    double s = sin(OR_PI * tau / g->t_env);
    return s * s;
  }
  double h = g->t_env / (double)(g->n_env + 3);
  double e = 0.0;
  for (int k = 0; k < g->n_env; k++) e += g->env[k] * cubic_bspline(tau / h - (double)k);
  return e;
}

static double laser_time(const or_config* g, double tau) {
  if (tau < 0.0 || tau > g->t_env) return 0.0;
  return g->a0 * envelope(g, tau) * sin(g->omega * tau + g->phase);
}

/* Incident magnetic field of the laser for component a of B at storage index
   (i, j, k).  A plane wave with unit direction n and electric field e has
   B = n x e (c = 1): along +x, E_y gives B_z = E_y and E_z gives B_y = -E_z;
   at an angle theta toward +y, the in-plane E (pol 1) gives B_z = |E| and
   E_z (pol 2) gives B_y = -cos(theta) E_z. */
static double b_incident(const or_ctx* c, int a, int64_t i, int64_t j, int64_t k, double t) {
  const or_config* g = &c->g;
  if (g->a0 == 0.0) return 0.0;
  int want = g->pol == 2 ? 1 : 2; /* pol y drives B_z, pol z drives B_y */
  if (a != want) return 0.0;
  double x = ((double)i + 0.5 * STAG_B[a][0]) * g->dx[0];
  if (g->angle != 0.0) {
    double y = c->nd > 1 ? ((double)j + 0.5 * STAG_B[a][1]) * g->dx[1] - g->yc : 0.0;
    double tau = t - g->t_delay - (x * cos(g->angle) + y * sin(g->angle));
    double e = laser_time(g, tau);
    return a == 2 ? e : -cos(g->angle) * e;
  }
  double prof = 1.0;
  if (g->waist > 0.0) {
    double r2 = 0.0;
    if (c->nd > 1) {
      double y = ((double)j + 0.5 * STAG_B[a][1]) * g->dx[1] - g->yc;
      r2 += y * y;
    }
    if (c->nd > 2) {
      double z = ((double)k + 0.5 * STAG_B[a][2]) * g->dx[2] - g->zc;
      r2 += z * z;
    }
    prof = exp(-r2 / (g->waist * g->waist));
  }
  double e = prof * laser_time(g, t - g->t_delay - x);
  return a == 2 ? e : -e;
}

/* B -= (dt/2) curl E over the interior */
static void b_half(or_ctx* c) {
  double h = 0.5 * c->g.dt;
  double ix = 1.0 / c->g.dx[0];
  double iy = c->nd > 1 ? 1.0 / c->g.dx[1] : 0.0;
  double iz = c->nd > 2 ? 1.0 / c->g.dx[2] : 0.0;
  int64_t di = 1, dj = c->nd > 1 ? c->st[0] : 0, dk = c->nd > 2 ? c->st[0] * c->st[1] : 0;
  for (int64_t k = 0; k < c->nn[2]; k++)
    for (int64_t j = 0; j < c->nn[1]; j++)
      for (int64_t i = 0; i < c->nn[0]; i++) {
        int64_t f = fidx(c, i, j, k);
        double *Ex = c->E[0], *Ey = c->E[1], *Ez = c->E[2];
        double cx = (Ez[f + dj] - Ez[f]) * iy - (Ey[f + dk] - Ey[f]) * iz;
        double cy = (Ex[f + dk] - Ex[f]) * iz - (Ez[f + di] - Ez[f]) * ix;
        double cz = (Ey[f + di] - Ey[f]) * ix - (Ex[f + dj] - Ex[f]) * iy;
        c->B[0][f] -= h * cx;
        c->B[1][f] -= h * cy;
        c->B[2][f] -= h * cz;
      }
}

/* E += dt (curl B - J) over the interior */
static void e_full(or_ctx* c) {
  double dt = c->g.dt;
  double ix = 1.0 / c->g.dx[0];
  double iy = c->nd > 1 ? 1.0 / c->g.dx[1] : 0.0;
  double iz = c->nd > 2 ? 1.0 / c->g.dx[2] : 0.0;
  int64_t di = 1, dj = c->nd > 1 ? c->st[0] : 0, dk = c->nd > 2 ? c->st[0] * c->st[1] : 0;
  for (int64_t k = 0; k < c->nn[2]; k++)
    for (int64_t j = 0; j < c->nn[1]; j++)
      for (int64_t i = 0; i < c->nn[0]; i++) {
        int64_t f = fidx(c, i, j, k);
        double *Bx = c->B[0], *By = c->B[1], *Bz = c->B[2];
        double cx = (Bz[f] - Bz[f - dj]) * iy - (By[f] - By[f - dk]) * iz;
        double cy = (Bx[f] - Bx[f - dk]) * iz - (Bz[f] - Bz[f - di]) * ix;
        double cz = (By[f] - By[f - di]) * ix - (Bx[f] - Bx[f - dj]) * iy;
        c->E[0][f] += dt * (cx - c->J[0][f]);
        c->E[1][f] += dt * (cy - c->J[1][f]);
        c->E[2][f] += dt * (cz - c->J[2][f]);
      }
}

/* periodic ghosts: E at index n copies index 0; B at index -1 copies n-1 */
static void periodic_e(or_ctx* c) {
  for (int d = 0; d < c->nd; d++) {
    if (!periodic(c, d)) continue;
    int64_t na, nb;
    face_extent(c, d, &na, &nb);
    for (int64_t b = 0; b < nb; b++)
      for (int64_t a = 0; a < na; a++) {
        int64_t i, j, k, i0, j0, k0;
        face_ijk(d, c->nn[d], a, b, &i, &j, &k);
        face_ijk(d, 0, a, b, &i0, &j0, &k0);
        for (int q = 0; q < 3; q++) c->E[q][fidx(c, i, j, k)] = c->E[q][fidx(c, i0, j0, k0)];
      }
  }
}
static void periodic_b(or_ctx* c) {
  for (int d = 0; d < c->nd; d++) {
    if (!periodic(c, d)) continue;
    int64_t na, nb;
    face_extent(c, d, &na, &nb);
    for (int64_t b = 0; b < nb; b++)
      for (int64_t a = 0; a < na; a++) {
        int64_t i, j, k, i0, j0, k0;
        face_ijk(d, -1, a, b, &i, &j, &k);
        face_ijk(d, c->nn[d] - 1, a, b, &i0, &j0, &k0);
        for (int q = 0; q < 3; q++) c->B[q][fidx(c, i, j, k)] = c->B[q][fidx(c, i0, j0, k0)];
      }
  }
}

/* First-order Mur condition at the low face of dim d, applied to the
   scattered part of the tangential B at the ghost node (half a cell
   outside), after the first B half step: B^{n+1/2}.  The ghost keeps its
   previous value (n-1/2); mur_b holds the first interior value at n-1/2. */
static void mur_low_b(or_ctx* c, int d) {
  double dt = c->g.dt, dx = c->g.dx[d];
  double kc = (dt - dx) / (dt + dx);
  int las = (d == 0 && c->g.bc_lo[0] == OR_LASER);
  double tn = (double)c->step * dt;
  double tm = tn - 0.5 * dt, tp = tn + 0.5 * dt;
  int t0, t1;
  tangential(d, &t0, &t1);
  int comps[2] = {t0, t1};
  int64_t na, nb;
  face_extent(c, d, &na, &nb);
  for (int q = 0; q < 2; q++) {
    int a_ = comps[q];
    double* Bf = c->B[a_];
    double* prev = c->mur_b[d][q];
    for (int64_t b = 0; b < nb; b++)
      for (int64_t a = 0; a < na; a++) {
        int64_t ig, jg, kg, i1, j1, k1;
        face_ijk(d, -1, a, b, &ig, &jg, &kg);
        face_ijk(d, 0, a, b, &i1, &j1, &k1);
        int64_t fg = fidx(c, ig, jg, kg), f1 = fidx(c, i1, j1, k1);
        double inc_g_m = 0, inc_g_p = 0, inc_1_m = 0, inc_1_p = 0;
        if (las) {
          inc_g_m = b_incident(c, a_, ig, jg, kg, tm);
          inc_g_p = b_incident(c, a_, ig, jg, kg, tp);
          inc_1_m = b_incident(c, a_, i1, j1, k1, tm);
          inc_1_p = b_incident(c, a_, i1, j1, k1, tp);
        }
        int64_t pi = a + na * b;
        double s1_old = prev[pi] - inc_1_m;
        double sg_old = Bf[fg] - inc_g_m;
        double s1_new = Bf[f1] - inc_1_p;
        double sg_new = s1_old + kc * (s1_new - sg_old);
        Bf[fg] = sg_new + inc_g_p;
        prev[pi] = Bf[f1];
      }
  }
}

static void save_high_e(or_ctx* c, int d) {
  int t0, t1;
  tangential(d, &t0, &t1);
  int comps[2] = {t0, t1};
  int64_t na, nb;
  face_extent(c, d, &na, &nb);
  for (int q = 0; q < 2; q++)
    for (int64_t b = 0; b < nb; b++)
      for (int64_t a = 0; a < na; a++) {
        int64_t i, j, k;
        face_ijk(d, c->nn[d] - 1, a, b, &i, &j, &k);
        c->mur_e[d][q][a + na * b] = c->E[comps[q]][fidx(c, i, j, k)];
      }
}

/* First-order Mur at the high face of dim d on the tangential E at the
   ghost node n (on the face), after the E update. */
static void mur_high_e(or_ctx* c, int d) {
  double dt = c->g.dt, dx = c->g.dx[d];
  double kc = (dt - dx) / (dt + dx);
  int t0, t1;
  tangential(d, &t0, &t1);
  int comps[2] = {t0, t1};
  int64_t na, nb;
  face_extent(c, d, &na, &nb);
  for (int q = 0; q < 2; q++)
    for (int64_t b = 0; b < nb; b++)
      for (int64_t a = 0; a < na; a++) {
        int64_t ig, jg, kg, i1, j1, k1;
        face_ijk(d, c->nn[d], a, b, &ig, &jg, &kg);
        face_ijk(d, c->nn[d] - 1, a, b, &i1, &j1, &k1);
        double* Ef = c->E[comps[q]];
        int64_t fg = fidx(c, ig, jg, kg), f1 = fidx(c, i1, j1, k1);
        Ef[fg] = c->mur_e[d][q][a + na * b] + kc * (Ef[f1] - Ef[fg]);
      }
}

static void field_step(or_ctx* c) {
  periodic_e(c);
  b_half(c);
  periodic_b(c);
  for (int d = 0; d < c->nd; d++)
    if (!periodic(c, d)) mur_low_b(c, d);
  for (int d = 0; d < c->nd; d++)
    if (!periodic(c, d)) save_high_e(c, d);
  e_full(c);
  periodic_e(c);
  for (int d = 0; d < c->nd; d++)
    if (!periodic(c, d)) mur_high_e(c, d);
  b_half(c);
  periodic_b(c);
}

/* ------------------------------------------------------------------- step */

static void record_probes(or_ctx* c) {
  if (c->nprobe == 0 || c->nrec >= c->g.max_probe_steps) return;
  for (int p = 0; p < c->nprobe; p++) {
    int q = c->pcomp[p];
    const int64_t* ix = &c->pidx[3 * p];
    double* F = q < 3 ? c->E[q] : c->B[q - 3];
    c->pdata[(int64_t)p * c->g.max_probe_steps + c->nrec] = F[fidx(c, ix[0], ix[1], ix[2])];
  }
  c->nrec++;
}

int or_set_probes(or_ctx* c, int nprobe, const int32_t* comp, const int64_t* idx3) {
  if (!c || nprobe < 0 || c->g.max_probe_steps <= 0) return -1;
  free(c->pcomp);
  free(c->pidx);
  free(c->pdata);
  c->nprobe = nprobe;
  c->pcomp = (int32_t*)calloc((size_t)nprobe + 1, sizeof(int32_t));
  c->pidx = (int64_t*)calloc((size_t)nprobe * 3 + 1, sizeof(int64_t));
  c->pdata = (double*)calloc((size_t)nprobe * c->g.max_probe_steps + 1, sizeof(double));
  for (int p = 0; p < nprobe; p++) {
    if (comp[p] < 0 || comp[p] > 5) return -1;
    c->pcomp[p] = comp[p];
    for (int d = 0; d < 3; d++) {
      int64_t v = idx3[3 * p + d];
      if (v < 0 || v >= c->nn[d]) return -1;
      c->pidx[3 * p + d] = v;
    }
  }
  c->nrec = 0;
  return 0;
}

int or_read_probes(or_ctx* c, double* out, int64_t* nrecorded) {
  if (!c) return -1;
  if (nrecorded) *nrecorded = c->nrec;
  if (out)
    for (int p = 0; p < c->nprobe; p++)
      for (int64_t t = 0; t < c->nrec; t++)
        out[(int64_t)p * c->nrec + t] = c->pdata[(int64_t)p * c->g.max_probe_steps + t];
  return 0;
}

static void charge_residual(or_ctx* c, const double* rho0, const double* rho1) {
  double dt = c->g.dt;
  double sum2 = 0.0, mx = 0.0, r2 = 0.0;
  for (int64_t k = 0; k < c->nn[2]; k++)
    for (int64_t j = 0; j < c->nn[1]; j++)
      for (int64_t i = 0; i < c->nn[0]; i++) {
        int64_t q = cidx(c, i, j, k);
        double drho = (rho1[q] - rho0[q]) / dt;
        double div = 0.0;
        int64_t ijk[3] = {i, j, k};
        for (int d = 0; d < c->nd; d++) {
          int64_t m[3] = {i, j, k};
          m[d] -= 1;
          double jm = 0.0;
          if (periodic(c, d)) {
            if (m[d] < 0) m[d] += c->nn[d];
            jm = c->J[d][fidx(c, m[0], m[1], m[2])];
          } else if (m[d] >= 0) {
            jm = c->J[d][fidx(c, m[0], m[1], m[2])];
          }
          div += (c->J[d][fidx(c, ijk[0], ijk[1], ijk[2])] - jm) / c->g.dx[d];
        }
        double res = drho + div;
        sum2 += res * res;
        r2 += drho * drho;
        if (fabs(res) > mx) mx = fabs(res);
      }
  c->div_l2 = sqrt(sum2);
  c->div_max = mx;
  c->rho_l2 = sqrt(r2);
}

int or_step(or_ctx* c, int nsteps) {
  if (!c || nsteps < 0) return -1;
  for (int it = 0; it < nsteps; it++) {
    int check = (c->g.flags & OR_CHARGE_CHECK) && it == nsteps - 1;
    double *rho0 = NULL, *rho1 = NULL;
    if (check) {
      rho0 = (double*)malloc((size_t)c->ncell * sizeof(double));
      rho1 = (double*)malloc((size_t)c->ncell * sizeof(double));
      or_rho(c, rho0);
    }
    for (int a = 0; a < 3; a++) memset(c->J[a], 0, (size_t)c->ntot * sizeof(double));
    for (int si = 0; si < c->nsp; si++) {
      or_species* s = &c->sp[si];
      for (int64_t p = 0; p < s->n; p++) {
        if (s->kind == OR_TWO_BODY)
          push_two_body(c, s, p);
        else if (s->kind == OR_MULTI_SHELL)
          push_multishell(c, s, p);
        else
          push_point(c, s, p);
      }
    }
    if (check) {
      or_rho(c, rho1);
      charge_residual(c, rho0, rho1);
      free(rho0);
      free(rho1);
    }
    if (!(c->g.flags & OR_FROZEN_FIELDS)) field_step(c);
    c->step++;
    record_probes(c);
  }
  return 0;
}

int or_diagnostics(or_ctx* c, or_diag* out) {
  if (!c || !out) return -1;
  memset(out, 0, sizeof(*out));
  out->step = c->step;
  out->time = (double)c->step * c->g.dt;
  double dV = 1.0;
  for (int d = 0; d < c->nd; d++) dV *= c->g.dx[d];
  double fe = 0.0;
  for (int64_t k = 0; k < c->nn[2]; k++)
    for (int64_t j = 0; j < c->nn[1]; j++)
      for (int64_t i = 0; i < c->nn[0]; i++) {
        int64_t f = fidx(c, i, j, k);
        for (int a = 0; a < 3; a++) fe += c->E[a][f] * c->E[a][f] + c->B[a][f] * c->B[a][f];
      }
  out->field_energy = 0.5 * fe * dV;
  double ke = 0.0, pm[3] = {0, 0, 0};
  int64_t np = 0;
  for (int si = 0; si < c->nsp; si++) {
    or_species* s = &c->sp[si];
    np += s->n;
    for (int64_t p = 0; p < s->n; p++) {
      double W = s->w ? s->w[p] : s->weight;
      const double* u1 = &s->u1[3 * p];
      double g1 = sqrt(1.0 + u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]);
      ke += W * s->m1 * (g1 - 1.0);
      for (int a = 0; a < 3; a++) pm[a] += W * s->m1 * u1[a];
      if (s->kind == OR_TWO_BODY) {
        const double* u2 = &s->u2[3 * p];
        double g2 = sqrt(1.0 + u2[0] * u2[0] + u2[1] * u2[1] + u2[2] * u2[2]);
        ke += W * s->m2 * (g2 - 1.0);
        for (int a = 0; a < 3; a++) pm[a] += W * s->m2 * u2[a];
      } else if (s->kind == OR_MULTI_SHELL) {
        for (int k = 0; k < s->nshell; k++) {
          const double* uk = &s->u2[3 * s->nshell * p + 3 * k];
          double gk = sqrt(1.0 + uk[0] * uk[0] + uk[1] * uk[1] + uk[2] * uk[2]);
          ke += W * s->mk[k] * (gk - 1.0);
          for (int a = 0; a < 3; a++) pm[a] += W * s->mk[k] * uk[a];
        }
      }
    }
  }
  out->kinetic_energy = ke;
  for (int a = 0; a < 3; a++) out->momentum[a] = pm[a];
  out->div_l2 = c->div_l2;
  out->div_max = c->div_max;
  out->rho_l2 = c->rho_l2;
  out->n_particles = np;
  out->error_word = c->err;
  return 0;
}
