// ctx.h -- host-side context of the library (shared by the C-ABI
// implementation and the gradient driver): species storage, the context
// struct, and the helpers that turn them into kernel arguments.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <string>
#include <vector>

#include "pic.h"
#include "pic_internal.h"
#include "shells.h"
#include "sort.h"
#include "tiled.h"

using pic::GridInfo;

struct GradState;  // gradient run: checkpoints, adjoint arrays (grad.hip)

struct SpeciesHost {
  pic_species_desc d{};
  double a_c = 0.0;  // softening length at the species' omega_c (inf: harmonic)
  bool ac_derived = false;  // a_c of each ion from its own omega_c (Sec. 3.1)
  int64_t n = 0, cap = 0;
  bool has_wc = false, has_w = false;
  double max_w = 0.0;  // largest |per-particle weight| loaded (has_w)
  void* cell = nullptr;
  void* off[3] = {nullptr, nullptr, nullptr};
  void* dl[3] = {nullptr, nullptr, nullptr};
  void* u1[3] = {nullptr, nullptr, nullptr};
  void* u2[3] = {nullptr, nullptr, nullptr};
  void* wc = nullptr;
  void* w = nullptr;
  // multi-shell ions: nshell clouds with their own charge, mass, bond
  // frequency and softening length; d_k and u_k per cloud (dl, u2 unused)
  int nshell = 0;
  double sq[pic::kMaxShell] = {}, sm[pic::kMaxShell] = {}, sw[pic::kMaxShell] = {},
         sa[pic::kMaxShell] = {};
  void* sdl[pic::kMaxShell][3] = {};
  void* su2[pic::kMaxShell][3] = {};
  pic::SortBuffers sort{};
  int64_t* ids = nullptr;  // device load indices (TRACK_IDS)
  uint32_t* outside = nullptr;  // particles listed as outside their tile (tiled kernel)
  bool needs_sort = true;  // tile offsets stale (after a load)
  // adaptive sort policy: particles advanced outside their tile since the
  // species' last sort, and steps since then
  double listed_since_sort = 0.0;
  int64_t steps_since_sort = 0;
};

// Species slots of the per-step outside-tile counters (device nslow[2 + s]).
constexpr int kMaxSpecies = 62;

struct pic_ctx {
  pic_config cfg{};
  pic_allocator alloc{};  // every device allocation of the context goes through it
  hipStream_t stream = nullptr;
  int device = 0;  // HIP device current at pic_create (the stream's device)
  GridInfo g{};
  int prec = 64;
  size_t rsize = 8;
  void* fields = nullptr;      // E, B: 6 planes (the present state)
  void* jfield = nullptr;      // J: 3 planes
  // the one-pass field step writes E, B and the low faces' Mur history to
  // a second set and the two sets swap roles after each step
  bool yee_fused = false;
  void* fields_alt = nullptr;  // 6 planes
  void* mur_b[3][2] = {};
  void* mur_b_alt[3][2] = {};
  void* mur_e[3][2] = {};
  uint32_t* err = nullptr;
  uint32_t* load_err = nullptr;
  uint32_t* nslow = nullptr;   // [0], [1]: list length scratch, [2 + s]: species s listed this step
  uint32_t* nfar = nullptr;    // [s]: ions of species s listed this step for their separation
  uint32_t* host_counts = nullptr;  // pinned: 2 slots of 128 (listed, then far) per-species counts
  hipEvent_t ev_counts[2] = {nullptr, nullptr};
  int counts_pending = -1;          // slot whose copy is in flight, or -1
  bool tiled = false;
  pic::TileGeom tg{};
  uint32_t* occ = nullptr;  // occupied-tile lists of sparse launches (tg.occ when in use)
  double* partials = nullptr;
  double* dout = nullptr;  // 32 doubles: [0..3] scratch, [4..6] residual, ...
  double* rho0 = nullptr;
  double* rho1 = nullptr;
  int nprobe = 0;
  int* probe_comp = nullptr;
  int64_t* probe_idx = nullptr;
  void* probe_buf = nullptr;
  int64_t probe_rec = 0;
  std::vector<std::unique_ptr<SpeciesHost>> sp;
  std::vector<void*> allocs;
  int64_t step = 0;
  int64_t steps_since_sort = 0;
  int tile[3] = {1, 1, 1};
  int ntiles[3] = {1, 1, 1};
  int sort_every = 0;  // > 0: fixed cadence; 0: adaptive per species
  std::string error;
  bool residual_valid = false;
  // timing
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_species;  // species of each (start, stop) pair
  size_t ev_used = 0;
  int64_t launches = 0;
  // gradient run (checkpoints and adjoint arrays), created on first use
  GradState* grad = nullptr;
  // bumped by every call that changes the state from outside a step
  // (loads, probes, species, pic_step); a gradient run records it
  uint64_t version = 0;
};

// Free the gradient run's host bookkeeping (its device buffers are in the
// context's allocation list).
void grad_release(pic_ctx* c);

// Record `msg` as the context's (or, without one, the creating thread's)
// last error and return `code`.
int fail(pic_ctx* c, int code, const std::string& msg);

#define HIPCHK(ctx, expr)                                                           \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return fail(ctx, PIC_EHIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

// Device memory from the caller's allocator (or hipMalloc), released at
// pic_destroy, or earlier by dev_release (synchronise the stream first).
void* dev_alloc(pic_ctx* c, size_t bytes);
void dev_release(pic_ctx* c, void* p);

inline bool is_periodic(const pic_config& c, int d) {
  return c.bc_lo[d] == PIC_BC_PERIODIC && c.bc_hi[d] == PIC_BC_PERIODIC;
}

template <typename Real>
pic::FieldPtrs<Real> field_ptrs(const pic_ctx* c) {
  pic::FieldPtrs<Real> f;
  Real* base = static_cast<Real*>(c->fields);
  Real* jb = static_cast<Real*>(c->jfield);
  for (int a = 0; a < 3; a++) {
    f.E[a] = base + (0 + a) * c->g.plane;
    f.B[a] = base + (3 + a) * c->g.plane;
    f.J[a] = jb + a * c->g.plane;
  }
  return f;
}

template <typename Real>
pic::SpeciesDev<Real> species_dev(const SpeciesHost& s) {
  pic::SpeciesDev<Real> d;
  d.cell = static_cast<uint32_t*>(s.cell);
  for (int a = 0; a < 3; a++) {
    d.off[a] = static_cast<Real*>(s.off[a]);
    d.dl[a] = static_cast<Real*>(s.dl[a]);
    d.u1[a] = static_cast<Real*>(s.u1[a]);
    d.u2[a] = static_cast<Real*>(s.u2[a]);
  }
  d.wc = s.has_wc ? static_cast<Real*>(s.wc) : nullptr;
  d.w = s.has_w ? static_cast<Real*>(s.w) : nullptr;
  d.n = s.n;
  return d;
}

template <typename Real>
pic::ShellDev<Real> shell_dev(const SpeciesHost& s) {
  pic::ShellDev<Real> d{};
  d.cell = static_cast<uint32_t*>(s.cell);
  for (int a = 0; a < 3; a++) {
    d.off[a] = static_cast<Real*>(s.off[a]);
    d.u0[a] = static_cast<Real*>(s.u1[a]);
    for (int k = 0; k < s.nshell; k++) {
      d.dl[k][a] = static_cast<Real*>(s.sdl[k][a]);
      d.uk[k][a] = static_cast<Real*>(s.su2[k][a]);
    }
  }
  d.w = s.has_w ? static_cast<Real*>(s.w) : nullptr;
  d.n = s.n;
  return d;
}

template <typename Real>
pic::ShellConst<Real> shell_const(const pic_ctx* c, const SpeciesHost& s) {
  pic::ShellConst<Real> k{};
  const int K = s.nshell;
  const double dt = c->cfg.dt, m0 = s.d.m1;
  double M = m0;
  for (int j = 0; j < K; j++) M += s.sm[j];
  auto body = [&](int b, double q, double m) {
    k.q[b] = (Real)q;
    k.inv_q[b] = (Real)(1.0 / q);
    k.m[b] = (Real)m;
    k.a[b] = (Real)(0.5 * dt * q / m);
    k.fm[b] = (Real)(m / M);
    k.qw[b] = (Real)(q * s.d.weight);
  };
  body(0, s.d.q1, m0);
  for (int j = 0; j < K; j++) {
    body(j + 1, s.sq[j], s.sm[j]);
    const double mp = m0 + s.sm[j];
    k.kap[j] = (Real)(m0 * s.sm[j] / mp * s.sw[j] * s.sw[j]);
    k.iac2[j] = std::isinf(s.sa[j]) ? Real(0) : (Real)(1.0 / (s.sa[j] * s.sa[j]));
    k.pf0[j] = (Real)(m0 / mp);
    k.pfk[j] = (Real)(s.sm[j] / mp);
    k.inv_mp[j] = (Real)(1.0 / mp);
  }
  k.inv_M = (Real)(1.0 / M);
  const double h = 0.5 * dt, nu = s.d.nu;
  k.D = (Real)((1.0 - nu * h) / (1.0 + nu * h));
  k.damp = nu > 0.0 ? 1 : 0;
  k.K = K;
  return k;
}

template <typename Real>
pic::PushConst<Real> push_const(const pic_ctx* c, const SpeciesHost& s) {
  pic::PushConst<Real> k{};
  const pic_species_desc& d = s.d;
  double dt = c->cfg.dt;
  bool two = d.kind == PIC_TWO_BODY;
  double m1 = d.m1, m2 = two ? d.m2 : 0.0, mc = m1 + m2;
  k.dt = (Real)dt;
  k.half_dt = (Real)(0.5 * dt);
  double dv = 1.0;
  for (int a = 0; a < 3; a++) {
    k.idx[a] = a < c->g.nd ? (Real)(1.0 / c->cfg.dx[a]) : Real(0);
    if (a < c->g.nd) dv *= c->cfg.dx[a];
  }
  k.a1 = (Real)(0.5 * dt * d.q1 / d.m1);
  k.a2 = two ? (Real)(0.5 * dt * d.q2 / d.m2) : Real(0);
  k.m1 = (Real)m1;
  k.m2 = (Real)m2;
  k.inv_mc = (Real)(1.0 / mc);
  k.f1 = two ? (Real)(m2 / mc) : Real(0);
  k.f2 = two ? (Real)(m1 / mc) : Real(1);
  k.mr = two ? (Real)(m1 * m2 / mc) : Real(0);
  k.inv_q1 = (Real)(1.0 / d.q1);
  k.inv_q2 = two ? (Real)(1.0 / d.q2) : Real(0);
  k.inv_ac2 = std::isinf(s.a_c) ? Real(0) : (Real)(1.0 / (s.a_c * s.a_c));
  // a_c^3 = C / omega_c^2 with C fixed: 1/a_c^2 = (omega_c^{4/3}) / C^{2/3}
  k.ac_k = two && s.ac_derived
               ? (Real)(1.0 / (s.a_c * s.a_c * std::pow(d.omega_c, 4.0 / 3.0)))
               : Real(0);
  k.omega_c = (Real)d.omega_c;
  k.nu = (Real)d.nu;
  k.nu_per_omega = (Real)d.nu_per_omega;
  k.qw1 = (Real)(d.q1 * d.weight);
  k.qw2 = two ? (Real)(d.q2 * d.weight) : Real(0);
  k.weight = (Real)d.weight;
  k.q1 = (Real)d.q1;
  k.q2 = two ? (Real)d.q2 : Real(0);
  for (int a = 0; a < 3; a++) k.jf[a] = a < c->g.nd ? (Real)(-c->cfg.dx[a] / (dt * dv)) : Real(0);
  for (int a = 0; a < 3; a++) k.dxs[a] = a < c->g.nd ? (Real)c->cfg.dx[a] : Real(0);
  k.inv_dv = (Real)(1.0 / dv);
  // Bound on one deposit term: charge x prefactor x shape factors.  The
  // running sum C of shape changes lies in [-1, 1]; the transverse factor
  // S0 (S0 + DS/2) + DS (S0/2 + DS/3) is at most 1 + 1/2; out-of-plane terms
  // carry |v| < c = 1 instead of C.  A merged pair adds both bodies.
  {
    const double wmax = s.has_w ? s.max_w : std::fabs(d.weight);
    const double qsum = (std::fabs(d.q1) + (two ? std::fabs(d.q2) : 0.0)) * wmax;
    double fmax = c->g.nd < 3 ? 1.0 / dv : 0.0;
    for (int a = 0; a < c->g.nd; a++) fmax = std::max(fmax, c->cfg.dx[a] / (dt * dv));
    const double bound = 1.5 * qsum * fmax;
    // no possible term (no weight yet): the largest scale, so that a shared
    // patch takes its partner species' scale
    int e = bound > 0.0 ? (int)std::floor(46.0 - std::log2(bound)) : 120;
    e = std::max(-120, std::min(120, e));
    k.jscale = (Real)std::ldexp(1.0, e);
  }
  k.two_body = two ? 1 : 0;
  k.deposit = (c->cfg.flags & PIC_FLAG_NO_DEPOSIT) ? 0 : 1;
  return k;
}

// Charge density of one species' bodies into the FP64 plane `rho`.
template <typename Real>
void launch_rho_species(const pic_ctx* c, const SpeciesHost& s, double* rho) {
  if (s.d.kind == PIC_MULTI_SHELL)
    pic::launch_rho_shells<Real>(c->g, shell_dev<Real>(s), shell_const<Real>(c, s),
                                 push_const<Real>(c, s), rho, c->stream);
  else if (c->tiled && !s.needs_sort && s.sort.tile_off)
    // sorted by tile: one LDS patch per tile (the offsets describe the
    // storage order until the next sort, wherever the particles moved)
    pic::launch_rho_tiled<Real>(c->g, species_dev<Real>(s), push_const<Real>(c, s),
                                s.sort.tile_off,
                                pic::TileGrid{{c->tile[0], c->tile[1], c->tile[2]},
                                              {c->ntiles[0], c->ntiles[1], c->ntiles[2]}},
                                rho, c->stream);
  else
    pic::launch_rho<Real>(c->g, species_dev<Real>(s), push_const<Real>(c, s), rho, c->stream);
}

// Laser description for the field kernels.
inline pic::LaserDev laser_dev(const pic_ctx* c) {
  const pic_laser& L = c->cfg.laser;
  pic::LaserDev las{};
  las.a0 = L.a0;
  las.omega = L.omega;
  las.t_env = L.t_env;
  las.waist = L.waist;
  las.yc = L.yc;
  las.zc = L.zc;
  las.phase = L.phase;
  las.t_delay = L.t_delay;
  las.pol = L.pol;
  las.on = (c->cfg.bc_lo[0] == PIC_BC_LASER && L.a0 != 0.0) ? 1 : 0;
  las.oblique = L.angle != 0.0 ? 1 : 0;
  las.cos_a = std::cos(L.angle);
  las.sin_a = std::sin(L.angle);
  las.n_env = L.n_env;
  las.h_env = L.n_env > 0 ? L.t_env / (double)(L.n_env + 3) : 0.0;
  for (int k = 0; k < 64; k++) las.env[k] = k < L.n_env ? L.env[k] : 0.0;
  return las;
}

// Allocate a species' per-particle omega_c / weight arrays (and their sort
// buffers) on the first load that brings them; fails once particles exist.
int prepare_optional(pic_ctx* c, SpeciesHost& s, bool want_wc, bool want_w);

// After the tile ranges changed (a sort, a restored state): choose dense or
// sparse tiled launches and rebuild the occupied-tile lists of the latter.
int update_occupancy(pic_ctx* c);

// Add the outside-tile counts of the last enqueued step to the sort policy
// (waits for that step's particle kernels).
void harvest_pending_counts(pic_ctx* c);

// Record a start (or stop) event of a timed particle-kernel dispatch with
// the given tag (species index; PIC_TIMING_ADJOINT + species for the
// adjoint kernel) when PIC_FLAG_TIMING is set.
bool record_event(pic_ctx* c, int tag, bool start);

// What one step does besides advancing the state.
struct StepOpts {
  bool check = false;   // charge-continuity residual of this step
  bool record = true;   // record the probes after the step
};

// Advance every species and the fields by one step (no tile sort); the
// state after the field guard fill and before the particle push is handed
// to `save` when given.
template <typename Real>
int advance_one(pic_ctx* c, const pic::LaserDev& las, const StepOpts& o,
                void (*save)(pic_ctx*, void*) = nullptr, void* save_arg = nullptr);
