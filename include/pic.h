/*
 * pic.h -- C ABI of libpic, the MI355X (gfx950) hot path of the two-body
 * macro-ion particle-in-cell method of An, Chen, Sheng and Zhang,
 * "Modeling of bound electron effects in particle-in-cell simulation"
 * (arXiv 2208.08038).
 *
 * One library call advances the whole per-step cycle on one GPU:
 *   tile sort -> field gather -> internal force + relativistic Boris push
 *   -> move -> Esirkepov current deposit -> Yee update with open (Mur)
 *   faces and laser injection -> optional FP64 diagnostics.
 *
 * Conventions shared by every entry point
 *  - Units are normalised: c = eps0 = e = m_e = 1 and laser angular
 *    frequency 1.  Lengths in c/omega, time in 1/omega, E in m_e c omega/e,
 *    B in m_e omega/e, charge in e, mass in m_e, momentum per mass u = p/(m c).
 *  - Every call returns pic_status (0 = PIC_OK, < 0 = error).  No C++
 *    exception crosses the ABI.  pic_last_error() returns a text for the
 *    last failure on a context (or of the last failed pic_create when ctx is
 *    NULL).
 *  - Host arrays passed in are read during the call and never retained;
 *    the caller keeps ownership.  Host arrays passed out are written during
 *    the call (the call synchronises the stream first).
 *  - All device memory comes from the caller's allocator (pic_allocator,
 *    required): the library never calls hipMalloc.  Memory is released
 *    through the allocator's free by pic_destroy.  (Pinned host memory for
 *    the asynchronous counter read-back is the library's own.)
 *  - Work is enqueued on the HIP stream given to pic_create.  pic_step is
 *    asynchronous; errors found on the device (non-finite state, particle
 *    out of range) surface at the next pic_diagnostics.  A context is not
 *    thread-safe; two contexts may run concurrently on different streams.
 *  - Field arrays exchanged with the host are FP64, component-major
 *    (3 planes of prod(n) interior values, x fastest, then y, then z).
 *    Component a of E sits half a cell up along axis a; component a of B
 *    sits half a cell up along the two other axes (Yee).
 */
#ifndef PIC_H
#define PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PIC_OK = 0,
  PIC_EINVAL = -1,  /* bad argument, shape, CFL violation, unsupported size */
  PIC_ENOMEM = -2,  /* allocator returned NULL or capacity exceeded */
  PIC_EHIP = -3,    /* HIP runtime error (text in pic_last_error) */
  PIC_ESTATE = -4,  /* call order misuse (e.g. particles before species) */
  PIC_ERANGE = -5,  /* particle outside the domain, the walls or the body range */
  PIC_ENAN = -6     /* non-finite particle state */
} pic_status;

/* boundary kinds per face */
#define PIC_BC_PERIODIC 0
#define PIC_BC_OPEN 1  /* first-order Mur absorbing face; particles (each body of a
                          two-body ion on its own) reflect `pad` cells inside */
#define PIC_BC_LASER 2 /* open face that also injects the laser (x-min only) */

/* configuration flags */
#define PIC_FLAG_FROZEN_FIELDS 1u /* skip the Maxwell update (fields stay as loaded) */
#define PIC_FLAG_NO_DEPOSIT 2u    /* push without depositing current */
#define PIC_FLAG_CHARGE_CHECK 4u  /* continuity residual of the last step of each pic_step */
#define PIC_FLAG_TRACK_IDS 8u     /* keep each particle's load index through sorts */
#define PIC_FLAG_TIMING 16u       /* time the particle kernels with HIP events */
#define PIC_FLAG_GLOBAL_KERNEL 32u /* advance particles from HBM with global atomics
                                      instead of the LDS-tiled kernel */
#define PIC_FLAG_SEPARATE_SPECIES 64u /* one tiled launch per species; by default a
                                         two-body and a point species (the only two
                                         species) share one launch per tile colour */

/* species kinds */
#define PIC_POINT 0
#define PIC_TWO_BODY 1
#define PIC_MULTI_SHELL 2 /* nucleus + 1..PIC_MAX_SHELL bound clouds (pic_add_multishell) */
#define PIC_MAX_SHELL 4

/* Device error word bits (pic_diag.error_word).  A macro-particle whose
   state is non-finite (NAN) or outside the representable range (RANGE: an
   offset outside [0, 1], or a body of a two-body ion outside the particle
   walls along a non-periodic axis) at the start of its cycle is left
   unchanged -- not advanced, no current -- and the bit is set.  One that
   leaves the range during its cycle (a jump of more than one node, a step
   out of the grid along a non-periodic axis) is advanced and flagged; it
   stops at its next cycle.  The particle walls mirror every body that
   reaches them, each body of a two-body ion on its own (with its momentum
   component reversed; the centre of mass and delta follow).  The bodies of
   a two-body ion may be any distance apart (Sec. 2: each body has its own
   position): an ion with a body outside [-1/2, 3/2) of the cell of its
   centre of mass (cell units) along a resolved axis is advanced from HBM
   with each body in the frame of the cell that holds it.  The bits stay set until the context is destroyed. */
#define PIC_ERR_NAN 1u
#define PIC_ERR_RANGE 2u

typedef struct {
  void* (*alloc)(size_t bytes, void* user); /* must return device memory aligned to 256 B */
  void (*free)(void* ptr, void* user);
  void* user;
} pic_allocator;

/* Laser entering through x-min (Sec. 3: x-ray pulse along +x):
   E_inc(x, t) = a0 sin^2(pi t'/t_env) sin(omega t' + phase) * G(y, z),
   t' = t - t_delay - x, nonzero for 0 <= t' <= t_env, G = exp(-r^2/waist^2)
   about (yc, zc) if waist > 0 else 1; pol 1 drives E_y (B_z = E_y),
   pol 2 drives E_z (B_y = -E_z).  angle != 0 (2D/3D, waist 0 only): a plane
   wave travelling at `angle` from +x toward +y, t' = t - t_delay -
   x cos(angle) - (y - yc) sin(angle); pol 1 keeps E in the x-y plane
   (B_z = |E|), pol 2 has E along z (B_y = -cos(angle) E_z).  With a periodic
   y axis the wave is periodic only if sin(angle) n_y dx_y omega / (2 pi) is
   an integer (the caller's choice).  n_env > 0 (at most PIC_MAX_ENV)
   replaces sin^2(pi t'/t_env) by the spline envelope
   sum_{k < n_env} env[k] N3(t'/h - k), h = t_env / (n_env + 3), N3 the
   cardinal cubic B-spline on [0, 4] (the envelope whose coefficients the
   gradient run differentiates). */
#define PIC_MAX_ENV 64
typedef struct {
  double a0, omega, t_env, waist, yc, zc, phase, t_delay;
  int32_t pol, reserved;
  double angle;
  int32_t n_env, reserved2;
  double env[PIC_MAX_ENV];
} pic_laser;

typedef struct {
  int32_t ndim;        /* 1, 2 or 3 resolved dimensions (x, x-y, x-y-z) */
  int32_t precision;   /* 32 or 64: particle state, fields and push arithmetic */
  int32_t pad;         /* particle walls sit pad (>= 3) cells inside non-periodic faces */
  int32_t max_probe_steps;
  int64_t n[3];        /* cells per resolved dimension; the packed cell index
                          needs sum_d ceil(log2 n_d) <= 31 */
  double dx[3];        /* cell sizes (resolved dimensions) */
  double dt;           /* must satisfy dt < 1/sqrt(sum_d dx_d^-2) */
  int32_t bc_lo[3], bc_hi[3];
  int32_t tile[3];     /* tile shape in cells (0: library default: 8x8x6 in 3D FP32,
                          8x8x8 in 3D FP64, 12x12 in 2D, 256 in 1D) */
  int32_t sort_every;  /* > 0: re-sort particles by tile every this many steps; 0: per
                          species, once the particles advanced outside their tile since
                          its last sort reach 1/200 of the species, or after 64 steps */
  uint32_t flags;
  int32_t reserved;
  double re_norm;      /* normalised classical electron radius 2 pi r_e / lambda */
  pic_laser laser;
} pic_config;

/* Species (Sec. 2).  Charges/masses are those of ONE real particle:
   two-body: nucleus q1, m1 and combined bound electron q2 = -Z_b, m2 = Z_b
   (q1 = q_c - q2, m1 = m_c - m2); point: q1, m1 only.  weight = real
   particles per macro-particle (in units of n_c (c/omega)^ndim); it scales
   only the deposited current, never the internal force.  omega_c (> 0) is
   the restoring frequency of Sec. 3.1; a_c the softening length: 0 derives
   a_c^3 = |q1 q2| re_norm / (m_r omega_c^2) (needs re_norm > 0), for each
   ion from its own omega_c when the particles carry one, since the Sec. 2
   potential has one Coulomb constant for all ions; +inf gives the harmonic
   bond; a finite a_c > 0 is used as given, and then the species' ions
   share its omega_c (per-particle omega_c is refused, PIC_EINVAL).
   Friction on the relative momentum: nu + nu_per_omega * omega_c. */
typedef struct {
  int32_t kind, reserved;
  double q1, m1, q2, m2;
  double weight, omega_c, a_c, nu, nu_per_omega;
  int64_t capacity;    /* maximum number of macro-particles */
} pic_species_desc;

typedef struct {
  int64_t step;
  double time;
  double field_energy;   /* 1/2 sum (E^2 + B^2) dV over interior nodes, FP64 compensated */
  double kinetic_energy; /* sum W m (gamma - 1) over bodies */
  double momentum[3];    /* sum W (m1 u1 + m2 u2) */
  double div_l2, div_max; /* (rho^{n+1} - rho^n)/dt + div J^{n+1/2} of the last step (CHARGE_CHECK) */
  double rho_l2;          /* L2 norm of (rho^{n+1} - rho^n)/dt */
  int64_t n_particles;
  uint32_t error_word, reserved;
  int64_t n_outside_tile; /* particles of the last step advanced outside their tile */
  int64_t n_far;          /* two-body ions of the last step with a body outside
                             [-1/2, 3/2) of their centre's cell (advanced from HBM,
                             each body in the frame of its own cell) */
} pic_diag;

typedef struct pic_ctx pic_ctx;

/* Create a simulation context.  cfg: grid, time step, boundaries, laser,
   flags.  alloc: device allocator (required; NULL or a NULL member:
   PIC_EINVAL, checked before any HIP call).  hip_stream: a
   hipStream_t (NULL: the null stream).  *out receives the context.
   Validates the CFL limit, sizes and boundary kinds (PIC_EINVAL). */
int pic_create(const pic_config* cfg, const pic_allocator* alloc, void* hip_stream,
               pic_ctx** out);

/* Add a species (Sec. 2 two-body macro-ion or point particle) with room for
   desc->capacity macro-particles; *species_id receives its id. */
int pic_add_species(pic_ctx* ctx, const pic_species_desc* desc, int32_t* species_id);

/* Add a multi-shell ion species: the bound electrons of an ion split into
   several components (the extension the paper's summary names), each cloud
   bound to the nucleus alone by the Sec. 2 bond.  desc: kind =
   PIC_MULTI_SHELL, q1 and m1 the nucleus, weight, nu (friction on each
   nucleus-cloud pair's relative momentum, applied pair by pair in shell
   order, pair momentum kept), capacity; the other fields are ignored.
   Cloud k < nshell (1..PIC_MAX_SHELL): charge shell_q[k] (!= 0), mass
   shell_m[k] > 0, restoring frequency shell_omega[k] > 0, softening length
   shell_ac[k] (0: derived as for a two-body ion, a^3 = |q1 q_k| re_norm /
   (m_r,k omega_k^2) with the pair's reduced mass m_r,k = m1 m_k / (m1 +
   m_k); +inf: harmonic; else as given).  One shell is exactly a two-body
   ion.  Particles (pic_load_particles or pic_load_particles_device): x =
   centre of mass of all bodies, delta n x 3 nshell (d_k = r_nucleus -
   r_cloud_k, shell k at 3k; NULL: 0), u1 the nucleus n x 3, u2 the clouds
   n x 3 nshell (NULL: every cloud moves with the nucleus), omega_c NULL
   (PIC_EINVAL otherwise); every body between the walls (PIC_ERANGE).
   pic_read_particles and pic_read_particles_range return delta and u2 with
   3 nshell values per particle.  The species is advanced one thread per
   ion, every body gathered and deposited in the frame of its own cell (in
   a tiled context, once sorted, with an LDS current patch per tile).
   Gradient runs refuse it (PIC_EINVAL). */
int pic_add_multishell(pic_ctx* ctx, const pic_species_desc* desc, int32_t nshell,
                       const double* shell_q, const double* shell_m, const double* shell_omega,
                       const double* shell_ac, int32_t* species_id);

/* Append n particles from HOST FP64 arrays:
   x      n x ndim physical positions (centre of mass r_c for two-body)
   delta  n x 3 relative displacement r1 - r2 (NULL: zero, the Sec. 2 start)
   u1     n x 3 momenta per mass; for a two-body species with u2 == NULL,
          u1 is the centre-of-mass momentum per mass u_c and the bodies get
          the Sec. 2 split p1 + p2 = m_c u_c, q1 v1 + q2 v2 = 0
   u2     n x 3 or NULL
   omega_c, weight: n values or NULL (species values); omega_c > 0 and only
          for a species whose a_c is derived or harmonic
   Positions are converted to (cell, offset) as xi = x/dx, cell = floor(xi),
   offset = xi - cell, then rounded to the context precision.  Particles
   are ordered by tile (stable).  PIC_ERANGE if outside the domain or the
   walls (two-body: either body outside the walls along a non-periodic
   axis); PIC_ENAN if non-finite, PIC_EINVAL for a bad omega_c, PIC_ENOMEM
   beyond capacity. */
int pic_load_particles(pic_ctx* ctx, int32_t species_id, int64_t n, const double* x,
                       const double* delta, const double* u1, const double* u2,
                       const double* omega_c, const double* weight);

/* Same contract as pic_load_particles, but every array is FP64 DEVICE
   memory on the context's device (read in stream order; the call
   synchronises before returning, after which the caller may free them).
   Conversion, the Sec. 2 split and the range checks run on the device; the
   whole species is then re-ordered by tile on the device (stable).  On an
   invalid particle nothing is appended and PIC_ERANGE / PIC_ENAN returns. */
int pic_load_particles_device(pic_ctx* ctx, int32_t species_id, int64_t n, const double* x,
                              const double* delta, const double* u1, const double* u2,
                              const double* omega_c, const double* weight);

/* Replace E and B from HOST FP64 interior arrays (layout above; NULL: zero). */
int pic_load_fields(pic_ctx* ctx, const double* E, const double* B);

/* Advance nsteps steps, asynchronously on the context stream. */
int pic_step(pic_ctx* ctx, int32_t nsteps);

/* FP64 diagnostics of the present state (synchronises).  Returns PIC_ENAN or
   PIC_ERANGE if the device error word is set (out is still filled). */
int pic_diagnostics(pic_ctx* ctx, pic_diag* out);

/* Copy E, B and the last step's J to HOST FP64 interior arrays (any may be NULL). */
int pic_read_fields(pic_ctx* ctx, double* E, double* B, double* J);

/* Number of particles in a species. */
int pic_count(pic_ctx* ctx, int32_t species_id, int64_t* n);

/* Copy a species' state to HOST arrays in the current device order:
   cell n x 3 int32 (per dimension, unused dims 0), offset n x 3, delta,
   u1, u2 n x 3 (delta/u2 two-body only), id n int64 load indices
   (PIC_FLAG_TRACK_IDS only).  Any pointer may be NULL. */
int pic_read_particles(pic_ctx* ctx, int32_t species_id, int32_t* cell, double* offset,
                       double* delta, double* u1, double* u2, int64_t* id);

/* The particles start .. start + count - 1 of a species in the library's
   present storage order (tile order after a sort; unchanged by a step that
   does not sort), same layouts as pic_read_particles, plus omega_c and
   weight (n each; the species value, resp. 1, where the species carries
   none).  Any pointer may be NULL.  PIC_EINVAL if the range is not inside
   the species.  Synchronises. */
int pic_read_particles_range(pic_ctx* ctx, int32_t species_id, int64_t start, int64_t count,
                             int32_t* cell, double* offset, double* delta, double* u1,
                             double* u2, double* omega_c, double* weight, int64_t* id);

/* Charge density at the integer nodes of the present state (HOST FP64, prod(n)). */
int pic_rho(pic_ctx* ctx, double* rho);

/* pic_rho without device scratch from the context, for callers that
   cannot allocate device memory at the time of the call (code under HIP
   graph capture, tight serving loops, harnesses that forbid allocation).
   Same result as pic_rho (to FP64 rounding: its atomics add in a varying
   order), computed in a static device array of 2^22 FP64 values (32 MiB;
   every GPU the library runs on holds its own copy until the process
   ends); the guarded grid, prod(n_d + 6) nodes over the resolved
   dimensions, must fit it (else PIC_EINVAL).  Calls no allocator: the
   context's device must be current (else PIC_ESTATE).  Calls on one GPU
   share the array, so calls that overlap on one GPU (two streams, two
   threads) race.  Synchronises. */
int pic_rho_static(pic_ctx* ctx, double* rho);

/* Field probes: component 0..5 (Ex, Ey, Ez, Bx, By, Bz) at interior node
   index (i, j, k), sampled after every step into a device buffer of
   max_probe_steps entries per probe.  Setting probes resets the record. */
int pic_set_probes(pic_ctx* ctx, int32_t nprobe, const int32_t* comp, const int64_t* ijk);
/* out: nprobe x nrecorded HOST FP64 (NULL: query *nrecorded only). */
int pic_read_probes(pic_ctx* ctx, double* out, int64_t* nrecorded);

/* Particle-kernel timing (PIC_FLAG_TIMING): total milliseconds and number
   of dispatches of the main particle-cycle kernel of one species
   (species_id >= 0) or of all species (-1) since the last reset, measured
   with HIP events recorded on the context stream around each dispatch.
   With the tiled kernel a species takes 2^ndim dispatches per step (one
   per tile colour), each timed on its own; the small kernel that advances
   particles found outside their tile is not included.  When a two-body
   and a point species share one launch per colour (the default for such a
   pair, see PIC_FLAG_SEPARATE_SPECIES), its dispatches count for the
   two-body species and none for the point species.  species_id =
   PIC_TIMING_ADJOINT + s selects the adjoint particle kernel of species s
   in gradient runs (one dispatch per reverse step).  Synchronises. */
#define PIC_TIMING_ADJOINT 65536
int pic_timing(pic_ctx* ctx, int32_t species_id, double* total_ms, int64_t* launches,
               int32_t reset);

/* Gradient run: the adjoint of the step (1D, 2D and 3D grids, both
   species kinds, FP32 and FP64), the differentiation axis that the bound-electron
   model of Sec. 2 / Sec. 3.1 opens: how a transmitted or reflected pulse
   depends on the restoring frequency omega_c, the friction rate and the
   laser's temporal envelope.

   pic_grad_forward advances the context by nsteps exactly as pic_step
   does, except that no tile sort runs during the run (the particles keep
   their storage order; a pending sort after a load runs first), recording
   the probes after every step, and keeps a device snapshot of the whole
   state every checkpoint_every steps (memory: ceil(nsteps / K) + K + 1
   snapshots, each the particle state plus E, B and the Mur history).
   Fails with PIC_EINVAL with PIC_FLAG_FROZEN_FIELDS or
   PIC_FLAG_NO_DEPOSIT, or when the probe record has no room for nsteps
   more steps.

   pic_grad_backward takes the cotangent of the probe values recorded by
   that run, dprobe[p * nsteps + n] = dL / d(probe p after step n of the
   run) (HOST FP64, nprobe x nsteps), and returns dL/d(parameter) for the
   parameters below, by re-running each checkpoint segment and reversing
   its steps (transposed Yee, Mur and guard operations; adjoint particle
   cycle).  Gradients with respect to omega_c are taken at fixed a_c (a
   derived a_c keeps the value fixed at pic_add_species); a species with
   per-particle omega_c gets the derivative with respect to a common shift
   of all of them; d_omega_c includes the nu_per_omega * omega_c part of
   the friction rate.  The context is left in the state at the end of the
   forward run, so pic_grad_backward may be called again with another
   cotangent.  Fails with PIC_ESTATE without a completed forward run, or
   once the context changed after it (pic_step, a load, new probes or
   species).  NULL outputs are skipped.  Synchronises. */
typedef struct {
  double* d_omega_c;  /* [number of species] */
  double* d_nu;       /* [number of species]: d/d(nu), the species' constant rate */
  double* d_env;      /* [laser.n_env]: d/d(env[k]) of the spline envelope */
  double* d_E;        /* 3 x ncell HOST FP64, layout of pic_load_fields: d/d(E at run start) */
  double* d_B;        /* same for B */
} pic_grad;
int pic_grad_forward(pic_ctx* ctx, int32_t nsteps, int32_t checkpoint_every);
int pic_grad_backward(pic_ctx* ctx, const double* dprobe, pic_grad* out);
/* After pic_grad_backward: dL/d(particle state at the start of the run)
   of one species, in the storage order of the run (the order
   pic_read_particles reports after pic_grad_forward; no sort runs during
   the run, but a sort pending from a load runs at its start): d_x
   (n x ndim, d/d position), d_delta, d_u1, d_u2 (n x 3; two-body only for
   delta and u2).  HOST FP64; NULL outputs are skipped. */
int pic_read_grad_particles(pic_ctx* ctx, int32_t species_id, double* d_x, double* d_delta,
                            double* d_u1, double* d_u2);

/* Checkpoint and restart.  pic_save_state writes the whole state that
   the following steps read -- E, B, the last step's J, the Mur history of
   the open faces, every species' particles in their storage order with the
   tile offsets of their last sort, per-particle omega_c and weight, load
   ids, the sort policy's counters, the step counter and the device error
   word -- into one HOST buffer: with host_buf NULL it only stores the size
   needed in *bytes; otherwise *bytes is the buffer's size on entry and the
   size written on return (PIC_EINVAL, with the size needed in *bytes, if it
   is too small).  Synchronises.  Probes (configuration, not state) and
   gradient runs are not saved.
   pic_load_state puts such a buffer back into a context created with the
   same pic_config (grid, precision, flags) and the same species (kinds,
   charges, masses) added in the same order, each with room for the
   state's particles; PIC_EINVAL if the buffer is not a state of such a
   context, PIC_ENOMEM if a species' capacity is too small.  The particles
   and fields the context held are replaced.  Run K steps, save, destroy,
   create, load and run N - K: the same state as N steps in one run (bit
   for bit wherever the run itself is: the FP32 fixed-point current with
   every particle in its tile; FP64 LDS and global atomics sum in a varying
   order).  The caller owns the buffer. */
int pic_save_state(pic_ctx* ctx, void* host_buf, size_t* bytes);
int pic_load_state(pic_ctx* ctx, const void* host_buf, size_t bytes);

/* Text of the last error on ctx (or of the last failed pic_create if NULL). */
const char* pic_last_error(const pic_ctx* ctx);

/* Release the context and all its device memory (synchronises first). */
void pic_destroy(pic_ctx* ctx);

/* Library version string. */
const char* pic_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PIC_H */
