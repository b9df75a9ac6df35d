/*
 * oracle.h -- plain FP64 CPU reference of the two-body macro-ion
 * particle-in-cell step (An, Chen, Sheng, Zhang, "Modeling of bound
 * electron effects in particle-in-cell simulation", arXiv 2208.08038).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this library: only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header or
 * constant with the HIP library; the two meet only through the seeded
 * input arrays.
 *
 * Units (normalised): c = eps0 = e = m_e = 1, omega_laser = 1.  Lengths in
 * c/omega, time in 1/omega, E in m_e c omega / e, B in m_e omega / e,
 * charge in e, mass in m_e, momentum per mass u = p/(m c).
 * Maxwell: dB/dt = -curl E, dE/dt = curl B - J.
 *
 * Particle positions are kept as an integer cell per resolved dimension
 * plus an offset in [0,1) in cell units.  A two-body macro-ion is stored as
 * its centre of mass R (cell + offset) and the relative displacement
 * delta = r1 - r2 (3 components, physical units), plus body momenta u1, u2
 * (Sec. 2: nucleus = body 1, combined bound electron = body 2).
 */
#ifndef PIC_ORACLE_H
#define PIC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_PERIODIC 0
#define OR_OPEN 1
#define OR_LASER 2 /* open face that also injects the laser; x-min only */

#define OR_FROZEN_FIELDS 1u /* no Maxwell update: fields stay as loaded */
#define OR_NO_DEPOSIT 2u    /* particles are pushed but deposit no current */
#define OR_CHARGE_CHECK 4u  /* compute rho before/after the last step of each or_step */

#define OR_MAX_ENV 64 /* largest number of envelope spline coefficients */

#define OR_POINT 0
#define OR_TWO_BODY 1
#define OR_MULTI_SHELL 2 /* nucleus + up to 4 bound clouds, each with its own bond */

/* error word bits */
#define OR_ERR_NAN 1u
#define OR_ERR_RANGE 2u

typedef struct {
  int32_t ndim;   /* 1, 2 or 3 resolved dimensions (x, then y, then z) */
  int32_t pol;    /* laser polarisation: 1 = E_y, 2 = E_z */
  int32_t pad;    /* particle walls sit `pad` cells inside every non-periodic face */
  int32_t max_probe_steps;
  int64_t n[3];   /* cells per resolved dimension (unused dims: 1) */
  double dx[3];   /* cell size per resolved dimension */
  double dt;
  int32_t bc_lo[3], bc_hi[3];
  uint32_t flags, reserved;
  /* laser entering at x-min: E_inc(t) = a0 * sin^2(pi t'/t_env) * sin(omega t' + phase),
     t' = t - t_delay - x, for 0 <= t' <= t_env; transverse Gaussian exp(-r^2/waist^2)
     about (yc, zc) when waist > 0, plane wave otherwise.  angle != 0 (2D and
     3D, plane wave only): the wave travels at `angle` from +x toward +y,
     t' = t - t_delay - x cos(angle) - (y - yc) sin(angle); pol 1 keeps E in
     the x-y plane (B along z), pol 2 has E along z.
     n_env > 0 replaces sin^2(pi t'/t_env) by the spline envelope
     sum_{k < n_env} env[k] N3(t'/h - k), h = t_env / (n_env + 3), with N3 the
     cardinal cubic B-spline supported on [0, 4]. */
  double a0, omega, t_env, waist, yc, zc, phase, t_delay, angle;
  int32_t n_env, reserved2;
  double env[OR_MAX_ENV];
} or_config;

typedef struct {
  int64_t step;
  double time;
  double field_energy;   /* 1/2 sum (E^2 + B^2) dV over the interior */
  double kinetic_energy; /* sum W m (gamma - 1) over bodies */
  double momentum[3];    /* sum W (m1 u1 + m2 u2) */
  double div_l2, div_max; /* charge-continuity residual of the last step (OR_CHARGE_CHECK) */
  double rho_l2;          /* L2 norm of (rho^{n+1}-rho^n)/dt, a scale for div_l2 */
  int64_t n_particles;
  uint32_t error_word, reserved;
} or_diag;

typedef struct or_ctx or_ctx;

or_ctx* or_create(const or_config* cfg);
void or_destroy(or_ctx* c);
/* Returns species id >= 0, or -1.  Two-body: omega_c > 0; a_c = 0 derives
   each ion's softening length from its own omega_c,
   a_c^3 = |q1 q2| re_norm / (m_r omega_c^2) (needs re_norm > 0); a_c = +inf
   is the harmonic bond; a finite a_c > 0 is used as given, and such a
   species takes no per-particle omega_c. */
int or_add_species(or_ctx* c, int kind, double q1, double m1, double q2, double m2,
                   double weight, double omega_c, double a_c, double nu, double nu_per_omega,
                   double re_norm, int64_t capacity);
/* Multi-shell ion: nucleus (q0, m0) and nshell (1..4) clouds, cloud k with
   charge qk[k], mass mk[k], bond frequency wk[k] and softening length ak[k]
   (0: derived as for a two-body ion with the pair's reduced mass; +inf:
   harmonic).  Particles: x = centre of mass of all bodies, delta = n*3*nshell
   (d_k = r_nucleus - r_cloud_k, shell k at 3k), u1 = nucleus n*3, u2 =
   clouds n*3*nshell (NULL: each cloud moves with the nucleus); no
   per-particle omega_c.  Returns species id >= 0, or -1. */
int or_add_multishell(or_ctx* c, double q0, double m0, int nshell, const double* qk,
                      const double* mk, const double* wk, const double* ak, double weight,
                      double nu, double re_norm, int64_t capacity);
/* Appends n particles.  x: n*ndim physical positions (centre of mass for
   two-body), delta: n*3 or NULL (= 0; any size: each body has its own
   position), u1: n*3, u2: n*3 or NULL.  For a
   two-body species with u2 == NULL, u1 is the centre-of-mass momentum per
   mass u_c and the Sec. 2 initial split is applied.  omega_c / weight:
   per-particle values or NULL (species value).  Returns 0 or <0. */
int or_load_particles(or_ctx* c, int sid, int64_t n, const double* x, const double* delta,
                      const double* u1, const double* u2, const double* omega_c,
                      const double* weight);
/* E, B: 3 component planes of prod(n) interior values each, x fastest. */
int or_load_fields(or_ctx* c, const double* E, const double* B);
int or_step(or_ctx* c, int nsteps);
int or_diagnostics(or_ctx* c, or_diag* out);
int or_read_fields(or_ctx* c, double* E, double* B, double* J);
/* cell: n*3 int32 (per dim), off: n*3, delta/u1/u2: n*3, multi-shell
   delta/u2 n*3*nshell (may be NULL) */
int or_read_particles(or_ctx* c, int sid, int32_t* cell, double* off, double* delta,
                      double* u1, double* u2);
int64_t or_count(or_ctx* c, int sid);
/* charge density at integer nodes (prod(n) values) for the present state */
int or_rho(or_ctx* c, double* rho);
/* field values at a position given as cell + offset (tests of the gather) */
int or_gather(or_ctx* c, const int32_t* cell, const double* off, double* E, double* B);
/* probes: component 0..5 (Ex,Ey,Ez,Bx,By,Bz) at interior index (i,j,k),
   sampled after every step */
int or_set_probes(or_ctx* c, int nprobe, const int32_t* comp, const int64_t* idx3);
int or_read_probes(or_ctx* c, double* out /* nprobe * nrecorded */, int64_t* nrecorded);
/* initial two-body split of a centre-of-mass momentum (Sec. 2) */
void or_split_momentum(double q1, double m1, double q2, double m2, const double* uc,
                       double* u1, double* u2);
/* softening length from the restoring frequency (Sec. 3.1): a_c^3 = |q1 q2| r_e / (m_r w_c^2) */
double or_ac_from_omega(double q1, double m1, double q2, double m2, double omega_c,
                        double re_norm);

#ifdef __cplusplus
}
#endif
#endif
