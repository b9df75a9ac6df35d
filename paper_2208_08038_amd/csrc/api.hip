// api.hip -- host implementation of the C ABI declared in include/pic.h:
// context and memory plan, particle loading (position -> cell + offset,
// Sec. 2 initial momentum split, tile ordering), the per-step launch
// schedule, diagnostics and read-back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <memory>
#include <string>
#include <vector>

#include "ctx.h"
#include "load.h"

namespace {

thread_local std::string g_create_error;

}  // namespace

int fail(pic_ctx* c, int code, const std::string& msg) {
  if (c)
    c->error = msg;
  else
    g_create_error = msg;
  return code;
}

// All device memory of a context comes from the caller's allocator.
void* dev_alloc(pic_ctx* c, size_t bytes) {
  if (bytes == 0) bytes = 256;
  bytes = (bytes + 255) & ~size_t(255);
  void* p = c->alloc.alloc(bytes, c->alloc.user);
  if (p) c->allocs.push_back(p);
  return p;
}

void dev_release(pic_ctx* c, void* p) {
  if (!p) return;
  auto it = std::find(c->allocs.begin(), c->allocs.end(), p);
  if (it == c->allocs.end()) return;
  c->allocs.erase(it);
  c->alloc.free(p, c->alloc.user);
}

namespace {

// pinned host buffer and events of the sort policy
void release_host(pic_ctx* c) {
  if (c->host_counts) (void)hipHostFree(c->host_counts);
  c->host_counts = nullptr;
  for (int t = 0; t < 2; t++) {
    if (c->ev_counts[t]) (void)hipEventDestroy(c->ev_counts[t]);
    c->ev_counts[t] = nullptr;
  }
}

void dev_free_all(pic_ctx* c) {
  for (void* p : c->allocs) c->alloc.free(p, c->alloc.user);
  c->allocs.clear();
}

int ceil_log2(int64_t n) {
  int b = 0;
  while ((int64_t(1) << b) < n) b++;
  return b;
}

// Sec. 2 initial split: m1 u1 + m2 u2 = m_c u_c with q1 v1 + q2 v2 = 0.
// Both velocities are parallel to u_c and v1 = alpha v2, alpha = -q2/q1;
// the speed s of body 2 solves g(s) = m1 alpha s gamma(alpha s) +
// m2 s gamma(s) - m_c |u_c| = 0, solved here by safeguarded Newton steps.
void split_momentum(double q1, double m1, double q2, double m2, const double* uc, double* u1,
                    double* u2) {
  double mc = m1 + m2;
  double p = std::sqrt(uc[0] * uc[0] + uc[1] * uc[1] + uc[2] * uc[2]);
  if (p == 0.0) {
    for (int a = 0; a < 3; a++) u1[a] = u2[a] = 0.0;
    return;
  }
  if (q1 + q2 == 0.0) {
    for (int a = 0; a < 3; a++) u1[a] = u2[a] = uc[a];
    return;
  }
  double al = -q2 / q1;
  double smax = std::fabs(al) > 1.0 ? 1.0 / std::fabs(al) : 1.0;
  double target = mc * p;
  double lo = 0.0, hi = smax;
  double s = std::min(target / (m1 * al + m2), 0.5 * smax);
  for (int it = 0; it < 100; it++) {
    double g1 = 1.0 / std::sqrt(1.0 - al * al * s * s), g2 = 1.0 / std::sqrt(1.0 - s * s);
    double gval = m1 * al * s * g1 + m2 * s * g2 - target;
    if (gval < 0)
      lo = s;
    else
      hi = s;
    double dg = m1 * al * g1 * g1 * g1 + m2 * g2 * g2 * g2;  // d/ds of s gamma(c s) = gamma^3
    double sn = s - gval / dg;
    if (!(sn > lo && sn < hi)) sn = 0.5 * (lo + hi);
    if (sn == s) break;
    s = sn;
  }
  double g2 = 1.0 / std::sqrt(1.0 - s * s);
  double g1 = 1.0 / std::sqrt(1.0 - al * al * s * s);
  for (int a = 0; a < 3; a++) {
    double e = uc[a] / p;
    u2[a] = g2 * s * e;
    u1[a] = g1 * al * s * e;
  }
}

template <typename Real>
int upload(pic_ctx* c, void* dst, const std::vector<Real>& v, int64_t at) {
  if (v.empty()) return PIC_OK;
  HIPCHK(c, hipMemcpyAsync(static_cast<Real*>(dst) + at, v.data(), v.size() * sizeof(Real),
                           hipMemcpyHostToDevice, c->stream));
  return PIC_OK;
}

template <typename Real>
int load_particles_t(pic_ctx* c, SpeciesHost& s, int64_t n, const double* x, const double* delta,
                     const double* u1, const double* u2, const double* wc, const double* w) {
  const int nd = c->g.nd;
  const bool two = s.d.kind == PIC_TWO_BODY;
  std::vector<uint32_t> cell(n);
  std::vector<int64_t> key(n);
  std::vector<double> off(n * 3, 0.0), du1(n * 3), du2(two ? n * 3 : 0), ddl(two ? n * 3 : 0);
  for (int64_t p = 0; p < n; p++) {
    int ci[3] = {0, 0, 0};
    for (int d = 0; d < nd; d++) {
      double xv = x[p * nd + d];
      if (!std::isfinite(xv)) return fail(c, PIC_ENAN, "non-finite particle position");
      double xi = xv / c->cfg.dx[d];
      double f = std::floor(xi);
      if (f < 0 || f >= (double)c->g.n[d])
        return fail(c, PIC_ERANGE, "particle position outside the grid");
      ci[d] = (int)f;
      double o = xi - f;
      if (!is_periodic(c->cfg, d)) {
        double pos = f + o;
        if (pos < (double)c->g.pad || pos > (double)(c->g.n[d] - c->g.pad))
          return fail(c, PIC_ERANGE, "particle outside the reflecting walls");
      }
      // round the offset to the working precision; an offset that rounds
      // up to 1 moves to the next cell (crossing rule)
      Real orr = (Real)o;
      if (orr >= Real(1)) {
        orr -= Real(1);
        ci[d] += 1;
        if (ci[d] >= c->g.n[d]) {
          if (is_periodic(c->cfg, d))
            ci[d] -= c->g.n[d];
          else
            return fail(c, PIC_ERANGE, "particle on the upper grid edge");
        }
      }
      off[p * 3 + d] = (double)orr;
    }
    uint32_t pk = (uint32_t)ci[0];
    if (nd > 1) pk |= (uint32_t)ci[1] << c->g.bits[0];
    if (nd > 2) pk |= (uint32_t)ci[2] << (c->g.bits[0] + c->g.bits[1]);
    cell[p] = pk;
    key[p] = (ci[0] / c->tile[0]) +
             (int64_t)c->ntiles[0] * ((ci[1] / c->tile[1]) + (int64_t)c->ntiles[1] * (ci[2] / c->tile[2]));
    const double* uu = u1 + 3 * p;
    for (int a = 0; a < 3; a++)
      if (!std::isfinite(uu[a])) return fail(c, PIC_ENAN, "non-finite momentum");
    if (two) {
      if (u2) {
        for (int a = 0; a < 3; a++) {
          du1[p * 3 + a] = uu[a];
          du2[p * 3 + a] = u2[3 * p + a];
          if (!std::isfinite(u2[3 * p + a])) return fail(c, PIC_ENAN, "non-finite momentum");
        }
      } else {
        split_momentum(s.d.q1, s.d.m1, s.d.q2, s.d.m2, uu, &du1[p * 3], &du2[p * 3]);
      }
      const double mc = s.d.m1 + s.d.m2;
      for (int a = 0; a < 3; a++) {
        double v = delta ? delta[3 * p + a] : 0.0;
        if (!std::isfinite(v)) return fail(c, PIC_ENAN, "non-finite delta");
        // along walled axes each body lies between the walls
        if (a < nd && !is_periodic(c->cfg, a)) {
          const double X = x[p * nd + a] / c->cfg.dx[a];
          const double X1 = X + (s.d.m2 / mc) * v / c->cfg.dx[a];
          const double X2 = X - (s.d.m1 / mc) * v / c->cfg.dx[a];
          const double lo = c->g.pad, hi = c->g.n[a] - c->g.pad;
          if (!(X1 >= lo && X1 <= hi && X2 >= lo && X2 <= hi))
            return fail(c, PIC_ERANGE, "a body of a two-body ion is outside the particle walls");
        }
        ddl[p * 3 + a] = v;
      }
      if (wc && !(wc[p] > 0))
        return fail(c, PIC_EINVAL, "per-particle omega_c must be positive");
    } else {
      for (int a = 0; a < 3; a++) du1[p * 3 + a] = uu[a];
    }
  }
  // stable order by tile (counting sort on the host)
  std::vector<int64_t> perm(n);
  {
    int64_t nt = (int64_t)c->ntiles[0] * c->ntiles[1] * c->ntiles[2];
    std::vector<int64_t> cnt(nt + 1, 0);
    for (int64_t p = 0; p < n; p++) cnt[key[p] + 1]++;
    for (int64_t t = 0; t < nt; t++) cnt[t + 1] += cnt[t];
    for (int64_t p = 0; p < n; p++) perm[cnt[key[p]]++] = p;
  }
  int64_t at = s.n;
  std::vector<uint32_t> hc(n);
  for (int64_t q = 0; q < n; q++) hc[q] = cell[perm[q]];
  HIPCHK(c, hipMemcpyAsync(static_cast<uint32_t*>(s.cell) + at, hc.data(), n * sizeof(uint32_t),
                           hipMemcpyHostToDevice, c->stream));
  std::vector<Real> buf(n);
  auto put = [&](void* dst, const std::vector<double>& src, int comp) -> int {
    for (int64_t q = 0; q < n; q++) buf[q] = (Real)src[perm[q] * 3 + comp];
    int rc = upload<Real>(c, dst, buf, at);
    if (rc) return rc;
    return hipStreamSynchronize(c->stream) == hipSuccess ? PIC_OK
                                                         : fail(c, PIC_EHIP, "sync failed");
  };
  int rc;
  for (int d = 0; d < nd; d++)
    if ((rc = put(s.off[d], off, d))) return rc;
  for (int a = 0; a < 3; a++) {
    if ((rc = put(s.u1[a], du1, a))) return rc;
    if (two) {
      if ((rc = put(s.u2[a], du2, a))) return rc;
      if ((rc = put(s.dl[a], ddl, a))) return rc;
    }
  }
  auto put1 = [&](void* dst, const double* src) -> int {
    for (int64_t q = 0; q < n; q++) buf[q] = (Real)src[perm[q]];
    int r = upload<Real>(c, dst, buf, at);
    if (r) return r;
    return hipStreamSynchronize(c->stream) == hipSuccess ? PIC_OK
                                                         : fail(c, PIC_EHIP, "sync failed");
  };
  if (wc || s.has_wc) {
    std::vector<double> tmp(n, s.d.omega_c);
    if (wc)
      for (int64_t p = 0; p < n; p++) tmp[p] = wc[p];
    if (!s.wc) return fail(c, PIC_ESTATE, "per-particle omega_c must come with the first load");
    if ((rc = put1(s.wc, tmp.data()))) return rc;
  }
  if (w || s.has_w) {
    std::vector<double> tmp(n, s.d.weight);
    if (w)
      for (int64_t p = 0; p < n; p++) tmp[p] = w[p];
    for (int64_t p = 0; p < n; p++) s.max_w = std::max(s.max_w, std::fabs(tmp[p]));
    if (!s.w) return fail(c, PIC_ESTATE, "per-particle weight must come with the first load");
    if ((rc = put1(s.w, tmp.data()))) return rc;
  }
  if (s.ids) {
    std::vector<int64_t> ids(n);
    for (int64_t q = 0; q < n; q++) ids[q] = at + perm[q];
    HIPCHK(c, hipMemcpyAsync(s.ids + at, ids.data(), n * sizeof(int64_t), hipMemcpyHostToDevice,
                             c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  s.n += n;
  s.needs_sort = true;
  return PIC_OK;
}

// Multi-shell load: x = centre of mass of all bodies, delta n x 3K (d_k =
// r_nucleus - r_cloud_k), u1 the nucleus, u2 n x 3K the clouds (NULL: every
// cloud moves with the nucleus); every body between the walls.
template <typename Real>
int load_shells_t(pic_ctx* c, SpeciesHost& s, int64_t n, const double* x, const double* delta,
                  const double* u1, const double* u2, const double* w) {
  const int nd = c->g.nd, K = s.nshell;
  double M = s.d.m1;
  for (int k = 0; k < K; k++) M += s.sm[k];
  std::vector<uint32_t> cell(n);
  std::vector<int64_t> key(n);
  std::vector<double> off(n * 3, 0.0), du0(n * 3), ddl(n * 3 * K), duk(n * 3 * K);
  for (int64_t p = 0; p < n; p++) {
    int ci[3] = {0, 0, 0};
    for (int d = 0; d < nd; d++) {
      double xv = x[p * nd + d];
      if (!std::isfinite(xv)) return fail(c, PIC_ENAN, "non-finite particle position");
      double xi = xv / c->cfg.dx[d];
      double f = std::floor(xi);
      if (f < 0 || f >= (double)c->g.n[d])
        return fail(c, PIC_ERANGE, "particle position outside the grid");
      ci[d] = (int)f;
      Real orr = (Real)(xi - f);
      if (orr >= Real(1)) {
        orr -= Real(1);
        ci[d] += 1;
        if (ci[d] >= c->g.n[d]) {
          if (is_periodic(c->cfg, d))
            ci[d] -= c->g.n[d];
          else
            return fail(c, PIC_ERANGE, "particle on the upper grid edge");
        }
      }
      off[p * 3 + d] = (double)orr;
    }
    for (int a = 0; a < 3 * K; a++) {
      const double v = delta ? delta[3 * K * p + a] : 0.0;
      if (!std::isfinite(v)) return fail(c, PIC_ENAN, "non-finite delta");
      ddl[3 * K * p + a] = v;
    }
    // along walled axes every body lies between the walls
    for (int d = 0; d < nd; d++) {
      if (is_periodic(c->cfg, d)) continue;
      double X0 = x[p * nd + d] / c->cfg.dx[d];
      for (int k = 0; k < K; k++) X0 += (s.sm[k] / M) * ddl[3 * K * p + 3 * k + d] / c->cfg.dx[d];
      const double lo = c->g.pad, hi = c->g.n[d] - c->g.pad;
      bool ok = X0 >= lo && X0 <= hi;
      for (int k = 0; k < K; k++) {
        const double Xk = X0 - ddl[3 * K * p + 3 * k + d] / c->cfg.dx[d];
        ok = ok && Xk >= lo && Xk <= hi;
      }
      if (!ok) return fail(c, PIC_ERANGE, "a body of a multi-shell ion is outside the particle walls");
    }
    for (int a = 0; a < 3; a++) {
      du0[3 * p + a] = u1[3 * p + a];
      if (!std::isfinite(u1[3 * p + a])) return fail(c, PIC_ENAN, "non-finite momentum");
    }
    for (int k = 0; k < K; k++)
      for (int a = 0; a < 3; a++) {
        const double v = u2 ? u2[3 * K * p + 3 * k + a] : u1[3 * p + a];
        if (!std::isfinite(v)) return fail(c, PIC_ENAN, "non-finite momentum");
        duk[3 * K * p + 3 * k + a] = v;
      }
    uint32_t pk = (uint32_t)ci[0];
    if (nd > 1) pk |= (uint32_t)ci[1] << c->g.bits[0];
    if (nd > 2) pk |= (uint32_t)ci[2] << (c->g.bits[0] + c->g.bits[1]);
    cell[p] = pk;
    key[p] = (ci[0] / c->tile[0]) +
             (int64_t)c->ntiles[0] * ((ci[1] / c->tile[1]) + (int64_t)c->ntiles[1] * (ci[2] / c->tile[2]));
  }
  std::vector<int64_t> perm(n);
  {
    int64_t nt = (int64_t)c->ntiles[0] * c->ntiles[1] * c->ntiles[2];
    std::vector<int64_t> cnt(nt + 1, 0);
    for (int64_t p = 0; p < n; p++) cnt[key[p] + 1]++;
    for (int64_t t = 0; t < nt; t++) cnt[t + 1] += cnt[t];
    for (int64_t p = 0; p < n; p++) perm[cnt[key[p]]++] = p;
  }
  const int64_t at = s.n;
  std::vector<uint32_t> hc(n);
  for (int64_t q = 0; q < n; q++) hc[q] = cell[perm[q]];
  HIPCHK(c, hipMemcpyAsync(static_cast<uint32_t*>(s.cell) + at, hc.data(), n * sizeof(uint32_t),
                           hipMemcpyHostToDevice, c->stream));
  std::vector<Real> buf(n);
  auto put = [&](void* dst, const std::vector<double>& src, int comp, int stride) -> int {
    for (int64_t q = 0; q < n; q++) buf[q] = (Real)src[perm[q] * stride + comp];
    int rc = upload<Real>(c, dst, buf, at);
    if (rc) return rc;
    return hipStreamSynchronize(c->stream) == hipSuccess ? PIC_OK
                                                         : fail(c, PIC_EHIP, "sync failed");
  };
  int rc;
  for (int d = 0; d < nd; d++)
    if ((rc = put(s.off[d], off, d, 3))) return rc;
  for (int a = 0; a < 3; a++)
    if ((rc = put(s.u1[a], du0, a, 3))) return rc;
  for (int k = 0; k < K; k++)
    for (int a = 0; a < 3; a++) {
      if ((rc = put(s.sdl[k][a], ddl, 3 * k + a, 3 * K))) return rc;
      if ((rc = put(s.su2[k][a], duk, 3 * k + a, 3 * K))) return rc;
    }
  if (w || s.has_w) {
    std::vector<double> tmp(n, s.d.weight);
    if (w)
      for (int64_t p = 0; p < n; p++) tmp[p] = w[p];
    for (int64_t p = 0; p < n; p++) s.max_w = std::max(s.max_w, std::fabs(tmp[p]));
    if (!s.w) return fail(c, PIC_ESTATE, "per-particle weight must come with the first load");
    if ((rc = put(s.w, tmp, 0, 1))) return rc;
  }
  if (s.ids) {
    std::vector<int64_t> ids(n);
    for (int64_t q = 0; q < n; q++) ids[q] = at + perm[q];
    HIPCHK(c, hipMemcpyAsync(s.ids + at, ids.data(), n * sizeof(int64_t), hipMemcpyHostToDevice,
                             c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  s.n += n;
  s.needs_sort = true;
  return PIC_OK;
}

// ------------------------------------------------------------ stepping

}  // namespace

// start/stop events around one particle-kernel launch (PIC_FLAG_TIMING)
constexpr size_t kMaxEvents = 1 << 16;
bool record_event(pic_ctx* c, int species, bool start) {
  if (!(c->cfg.flags & PIC_FLAG_TIMING)) return false;
  if (start && c->ev_used + 2 > kMaxEvents) return false;
  if (c->ev_used >= c->ev.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return false;
    c->ev.push_back(e);
  }
  if (start) {
    if (c->ev_species.size() < c->ev_used / 2 + 1) c->ev_species.resize(c->ev_used / 2 + 1);
    c->ev_species[c->ev_used / 2] = species;
  }
  return hipEventRecord(c->ev[c->ev_used++], c->stream) == hipSuccess;
}

namespace {

// timing events around each dispatch of the main particle kernel of one
// species (every colour of the tiled kernel; the outside-tile list kernel
// is not timed)
struct TimedDispatch {
  pic_ctx* c;
  int species;
  bool open;
  static void hook(void* arg, bool start) {
    auto* t = static_cast<TimedDispatch*>(arg);
    if (start) {
      t->open = record_event(t->c, t->species, true);
    } else if (t->open) {
      record_event(t->c, t->species, false);
      t->open = false;
    }
  }
};

// Add the outside-tile counts of the last enqueued step (waits for that
// step's particle kernels; the field update of the step may still run).
void harvest_counts(pic_ctx* c) {
  if (c->counts_pending < 0) return;
  const int slot = c->counts_pending;
  c->counts_pending = -1;
  if (hipEventSynchronize(c->ev_counts[slot]) != hipSuccess) return;
  // ions listed only for their separation stay listed after a sort: they
  // do not count toward the next one
  for (size_t si = 0; si < c->sp.size(); si++) {
    const uint32_t listed = c->host_counts[128 * slot + si];
    const uint32_t far = c->host_counts[128 * slot + 64 + si];
    c->sp[si]->listed_since_sort += (double)(listed >= far ? listed - far : 0u);
  }
}

template <typename Real>
void deposit_rho(pic_ctx* c, double* rho) {
  pic::launch_zero<double>(rho, c->g.plane, c->stream);
  for (auto& s : c->sp) launch_rho_species<Real>(c, *s, rho);
  pic::launch_fold_periodic_f64(c->g, rho, c->stream);
}

// Tile sort of each species that needs one: always after a load; then on
// a fixed cadence, or per species when the particles it advanced outside
// their tile since its last sort reach kSortRatio of the species (the
// outside-tile kernel costs about 1 / kSortRatio as much per particle as a
// sort does; the rule spends on sorting what the detour cost, so stays
// within twice the best cadence), or after kSortMaxSteps steps.  The sort
// after a load also orders each tile by rank within cell; later sorts are
// stable and keep that order for the particles that stayed.
int sort_due(pic_ctx* c) {
  constexpr double kSortRatio = 1.0 / 200.0;
  constexpr int64_t kSortMaxSteps = 64;
  if (c->sort_every == 0) harvest_counts(c);
  const bool cadence = c->sort_every > 0 && c->steps_since_sort >= c->sort_every;
  bool sorted = false;
  for (auto& s : c->sp) {
    bool due = cadence || s->needs_sort;
    if (c->sort_every == 0)
      due = due || s->listed_since_sort >= kSortRatio * (double)s->n ||
            s->steps_since_sort >= kSortMaxSteps;
    if (!due) continue;
    // the first sort after a host load also rebuilds the order within tiles
    int rc = pic::sort_by_tile(c->g, c->tile, c->ntiles, s->sort, s->n, c->stream,
                               s->needs_sort);
    if (rc) return fail(c, PIC_EHIP, "tile sort launch failed");
    s->needs_sort = false;
    s->listed_since_sort = 0.0;
    s->steps_since_sort = 0;
    sorted = true;
  }
  if (cadence) c->steps_since_sort = 0;
  return sorted ? update_occupancy(c) : PIC_OK;
}

}  // namespace

template <typename Real>
int advance_one(pic_ctx* c, const pic::LaserDev& las, const StepOpts& o,
                void (*save)(pic_ctx*, void*), void* save_arg) {
  const GridInfo& g = c->g;
  pic::FieldPtrs<Real> f = field_ptrs<Real>(c);
  Real* eb[6] = {f.E[0], f.E[1], f.E[2], f.B[0], f.B[1], f.B[2]};
  Real* jj[3] = {f.J[0], f.J[1], f.J[2]};
  const bool frozen = (c->cfg.flags & PIC_FLAG_FROZEN_FIELDS) != 0;
  const bool check = o.check;
  pic::launch_fill_periodic<Real>(g, eb, 6, c->stream);
  if (save) save(c, save_arg);
  pic::launch_zero<Real>(f.J[0], 3 * g.plane, c->stream);
  if (check) deposit_rho<Real>(c, c->rho0);
  if (c->tiled) {
    HIPCHK(c, hipMemsetAsync(c->nslow + 1, 0, 63 * sizeof(uint32_t), c->stream));
    HIPCHK(c, hipMemsetAsync(c->nfar, 0, 64 * sizeof(uint32_t), c->stream));
  }
  // a two-body and a point species share one tiled launch per tile colour
  // (one field staging and one current flush per tile for both)
  int pi = -1, pe = -1;
  if (c->tiled && c->sp.size() == 2 && !(c->cfg.flags & PIC_FLAG_SEPARATE_SPECIES)) {
    for (int q = 0; q < 2; q++)
      if (c->sp[q]->d.kind == PIC_TWO_BODY && c->sp[1 - q]->d.kind == PIC_POINT) {
        pi = q;
        pe = 1 - q;
      }
  }
  if (pi >= 0) {
    auto& si = c->sp[pi];
    auto& se = c->sp[pe];
    pic::PushConst<Real> ci = push_const<Real>(c, *si), ce = push_const<Real>(c, *se);
    ci.jscale = ce.jscale = std::min(ci.jscale, ce.jscale);  // one patch scale
    TimedDispatch td{c, pi, false};
    pic::DispatchHook hook;
    if (c->cfg.flags & PIC_FLAG_TIMING) hook = {&TimedDispatch::hook, &td};
    hipError_t e = pic::launch_push_tiled_pair<Real>(
        g, f, species_dev<Real>(*si), ci, si->sort.tile_off, si->outside, si->sort.key[0],
        species_dev<Real>(*se), ce, se->sort.tile_off, se->outside, c->tg, c->nslow,
        c->nslow + 2 + pi,
        c->nslow + 2 + pe, c->nfar + pi, c->err, c->stream, hook);
    if (e != hipSuccess)
      return fail(c, PIC_EHIP, std::string("tiled particle kernel: ") + hipGetErrorString(e));
    c->launches++;
    si->steps_since_sort++;
    se->steps_since_sort++;
  }
  for (size_t si = 0; si < c->sp.size() && pi < 0; si++) {
    auto& s = c->sp[si];
    TimedDispatch td{c, (int)si, false};
    if (s->d.kind == PIC_MULTI_SHELL) {
      // multi-shell ions: one thread per ion; once the species is sorted by
      // tile, one workgroup per tile with an LDS current patch (the 3D
      // two-cloud medium: FP32 3.72 -> 2.76 ms per step, FP64 6.75 -> 4.55)
      TimedDispatch::hook(&td, true);
      hipError_t e;
      const pic::TileGrid tgrid{{c->tile[0], c->tile[1], c->tile[2]},
                                {c->ntiles[0], c->ntiles[1], c->ntiles[2]}};
      if (c->tiled && !s->needs_sort && s->sort.tile_off &&
          pic::shells_tiled_lds(g, tgrid) <= pic::kShellsTiledMaxLds)
        e = pic::launch_push_shells_tiled<Real>(
            g, f, shell_dev<Real>(*s), shell_const<Real>(c, *s), push_const<Real>(c, *s),
            s->sort.tile_off, tgrid, c->err, c->stream);
      else
        e = pic::launch_push_shells<Real>(g, f, shell_dev<Real>(*s), shell_const<Real>(c, *s),
                                          push_const<Real>(c, *s), c->err, c->stream);
      TimedDispatch::hook(&td, false);
      if (e != hipSuccess)
        return fail(c, PIC_EHIP, std::string("multi-shell kernel: ") + hipGetErrorString(e));
    } else if (c->tiled) {
      pic::DispatchHook hook;
      if (c->cfg.flags & PIC_FLAG_TIMING) hook = {&TimedDispatch::hook, &td};
      hipError_t e = pic::launch_push_tiled<Real>(g, f, species_dev<Real>(*s),
                                                  push_const<Real>(c, *s), c->tg,
                                                  s->sort.tile_off, s->outside,
                                                  s->sort.key[0], c->nslow, c->nslow + 2 + si,
                                                  c->nfar + si, c->err, c->stream, hook);
      if (e != hipSuccess)
        return fail(c, PIC_EHIP, std::string("tiled particle kernel: ") + hipGetErrorString(e));
    } else {
      TimedDispatch::hook(&td, true);
      pic::launch_push<Real>(g, f, species_dev<Real>(*s), push_const<Real>(c, *s), c->err,
                             c->stream);
      TimedDispatch::hook(&td, false);
    }
    c->launches++;
    s->steps_since_sort++;
  }
  // the step's outside-tile counts go to pinned host memory, read before
  // the next step is enqueued
  if (c->tiled && c->sort_every == 0 && !c->sp.empty()) {
    const int slot = (int)(c->step & 1);
    HIPCHK(c, hipMemcpyAsync(c->host_counts + 128 * slot, c->nslow + 2,
                             c->sp.size() * sizeof(uint32_t), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipMemcpyAsync(c->host_counts + 128 * slot + 64, c->nfar,
                             c->sp.size() * sizeof(uint32_t), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipEventRecord(c->ev_counts[slot], c->stream));
    c->counts_pending = slot;
  }
  pic::launch_fold_periodic<Real>(g, jj, 3, c->stream);
  if (check) {
    deposit_rho<Real>(c, c->rho1);
    pic::launch_residual<Real>(g, f, c->rho0, c->rho1, c->partials, pic::reduce_blocks(),
                               c->dout + 4, c->stream);
    c->residual_valid = true;
  }
  if (!frozen && c->yee_fused) {
    pic::FieldPtrs<Real> fo = f;
    Real* ob = static_cast<Real*>(c->fields_alt);
    for (int a = 0; a < 3; a++) {
      fo.E[a] = ob + a * g.plane;
      fo.B[a] = ob + (3 + a) * g.plane;
    }
    Real* hin[3][2] = {};
    Real* hout[3][2] = {};
    for (int d = 0; d < 3; d++)
      for (int t = 0; t < 2; t++) {
        hin[d][t] = static_cast<Real*>(c->mur_b[d][t]);
        hout[d][t] = static_cast<Real*>(c->mur_b_alt[d][t]);
      }
    hipError_t e = pic::launch_yee_fused<Real>(g, f, fo, hin, hout, las, c->step, c->stream);
    if (e != hipSuccess)
      return fail(c, PIC_EHIP, std::string("field step: ") + hipGetErrorString(e));
    std::swap(c->fields, c->fields_alt);
    for (int d = 0; d < 3; d++)
      for (int t = 0; t < 2; t++) std::swap(c->mur_b[d][t], c->mur_b_alt[d][t]);
    f = field_ptrs<Real>(c);
  } else if (!frozen) {
    pic::launch_b_half<Real>(g, f, c->stream);
    pic::launch_fill_periodic<Real>(g, eb + 3, 3, c->stream);
    for (int d = 0; d < g.nd; d++)
      if (!g.periodic[d])
        pic::launch_mur_low_b<Real>(g, f, d, static_cast<Real*>(c->mur_b[d][0]),
                                    static_cast<Real*>(c->mur_b[d][1]), las, c->step,
                                    c->stream);
    for (int d = 0; d < g.nd; d++)
      if (!g.periodic[d])
        pic::launch_save_high_e<Real>(g, f, d, static_cast<Real*>(c->mur_e[d][0]),
                                      static_cast<Real*>(c->mur_e[d][1]), c->stream);
    pic::launch_e_full<Real>(g, f, c->stream);
    pic::launch_fill_periodic<Real>(g, eb, 3, c->stream);
    for (int d = 0; d < g.nd; d++)
      if (!g.periodic[d])
        pic::launch_mur_high_e<Real>(g, f, d, static_cast<Real*>(c->mur_e[d][0]),
                                     static_cast<Real*>(c->mur_e[d][1]), c->stream);
    pic::launch_b_half<Real>(g, f, c->stream);
  }
  c->step++;
  c->steps_since_sort++;
  if (o.record && c->nprobe > 0 && c->probe_rec < c->cfg.max_probe_steps) {
    pic::launch_probes<Real>(g, f, c->nprobe, c->probe_comp, c->probe_idx,
                             static_cast<Real*>(c->probe_buf), c->cfg.max_probe_steps,
                             c->probe_rec, c->stream);
    c->probe_rec++;
  }
  return PIC_OK;
}

template int advance_one<float>(pic_ctx*, const pic::LaserDev&, const StepOpts&,
                                void (*)(pic_ctx*, void*), void*);
template int advance_one<double>(pic_ctx*, const pic::LaserDev&, const StepOpts&,
                                 void (*)(pic_ctx*, void*), void*);

namespace {

template <typename Real>
int step_t(pic_ctx* c, int nsteps) {
  const pic::LaserDev las = laser_dev(c);
  for (int it = 0; it < nsteps; it++) {
    int rc = sort_due(c);
    if (rc) return rc;
    StepOpts o;
    o.check = (c->cfg.flags & PIC_FLAG_CHARGE_CHECK) && it == nsteps - 1;
    rc = advance_one<Real>(c, las, o);
    if (rc) return rc;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, PIC_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return PIC_OK;
}

template <typename Real>
int diagnostics_t(pic_ctx* c, pic_diag* out) {
  pic::FieldPtrs<Real> f = field_ptrs<Real>(c);
  int nb = pic::reduce_blocks();
  pic::launch_field_energy<Real>(c->g, f, c->partials, nb, c->dout + 0, c->stream);
  double host[8];
  HIPCHK(c, hipMemcpyAsync(host, c->dout, 8 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double dv = 1.0;
  for (int d = 0; d < c->g.nd; d++) dv *= c->cfg.dx[d];
  std::memset(out, 0, sizeof(*out));
  out->field_energy = 0.5 * host[0] * dv;
  if (c->residual_valid) {
    out->div_l2 = std::sqrt(host[4]);
    out->div_max = host[5];
    out->rho_l2 = std::sqrt(host[6]);
  }
  double ke = 0.0, pm[3] = {0, 0, 0};
  int64_t np = 0;
  for (auto& sp : c->sp) {
    const SpeciesHost& s = *sp;
    np += s.n;
    if (s.n == 0) continue;
    // a multi-shell ion sums as its nucleus and each cloud, each viewed as
    // a point species of its own mass
    const int nbody = s.d.kind == PIC_MULTI_SHELL ? 1 + s.nshell : 1;
    for (int b = 0; b < nbody; b++) {
      pic::SpeciesDev<Real> sd = species_dev<Real>(s);
      pic::PushConst<Real> pc = push_const<Real>(c, s);
      if (s.d.kind == PIC_MULTI_SHELL) {
        pc.two_body = 0;
        pc.m1 = (Real)(b == 0 ? s.d.m1 : s.sm[b - 1]);
        if (b > 0)
          for (int a = 0; a < 3; a++) sd.u1[a] = static_cast<Real*>(s.su2[b - 1][a]);
      }
      pic::launch_kinetic<Real>(sd, pc, c->partials, nb, c->dout + 0, c->stream);
      double k4[4];
      HIPCHK(c, hipMemcpyAsync(k4, c->dout, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      ke += k4[0];
      for (int a = 0; a < 3; a++) pm[a] += k4[1 + a];
    }
  }
  uint32_t ew = 0, nsl[kMaxSpecies] = {}, nfr[kMaxSpecies] = {};
  HIPCHK(c, hipMemcpyAsync(&ew, c->err, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(nsl, c->nslow + 2, kMaxSpecies * sizeof(uint32_t),
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(nfr, c->nfar, kMaxSpecies * sizeof(uint32_t), hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  int64_t ns = 0, nf = 0;
  for (size_t si = 0; si < c->sp.size(); si++) {
    ns += nsl[si];
    nf += nfr[si];
  }
  out->step = c->step;
  out->time = (double)c->step * c->cfg.dt;
  out->kinetic_energy = ke;
  for (int a = 0; a < 3; a++) out->momentum[a] = pm[a];
  out->n_particles = np;
  out->error_word = ew;
  out->n_outside_tile = c->tiled ? (int64_t)ns : 0;
  out->n_far = c->tiled ? (int64_t)nf : 0;
  if (ew & PIC_ERR_NAN) return fail(c, PIC_ENAN, "non-finite particle state on the device");
  if (ew & PIC_ERR_RANGE) return fail(c, PIC_ERANGE, "particle out of range on the device");
  return PIC_OK;
}

template <typename Real>
int read_fields_t(pic_ctx* c, double* E, double* B, double* J) {
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const GridInfo& g = c->g;
  std::vector<Real> plane(g.plane);
  int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
  double* outs[9] = {E, E ? E + ncell : nullptr, E ? E + 2 * ncell : nullptr,
                     B, B ? B + ncell : nullptr, B ? B + 2 * ncell : nullptr,
                     J, J ? J + ncell : nullptr, J ? J + 2 * ncell : nullptr};
  for (int comp = 0; comp < 9; comp++) {
    if (!outs[comp]) continue;
    const Real* src = comp < 6 ? static_cast<Real*>(c->fields) + comp * g.plane
                               : static_cast<Real*>(c->jfield) + (comp - 6) * g.plane;
    HIPCHK(c, hipMemcpy(plane.data(), src, g.plane * sizeof(Real), hipMemcpyDeviceToHost));
    for (int k = 0; k < g.n[2]; k++)
      for (int j = 0; j < g.n[1]; j++)
        for (int i = 0; i < g.n[0]; i++)
          outs[comp][i + (int64_t)g.n[0] * (j + (int64_t)g.n[1] * k)] =
              (double)plane[g.origin + i + j * g.sy + k * g.sz];
  }
  return PIC_OK;
}

template <typename Real>
int load_fields_t(pic_ctx* c, const double* E, const double* B) {
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const GridInfo& g = c->g;
  std::vector<Real> plane(g.plane);
  int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
  for (int comp = 0; comp < 6; comp++) {
    const double* src = comp < 3 ? (E ? E + comp * ncell : nullptr)
                                 : (B ? B + (comp - 3) * ncell : nullptr);
    std::fill(plane.begin(), plane.end(), Real(0));
    if (src)
      for (int k = 0; k < g.n[2]; k++)
        for (int j = 0; j < g.n[1]; j++)
          for (int i = 0; i < g.n[0]; i++)
            plane[g.origin + i + j * g.sy + k * g.sz] =
                (Real)src[i + (int64_t)g.n[0] * (j + (int64_t)g.n[1] * k)];
    HIPCHK(c, hipMemcpy(static_cast<Real*>(c->fields) + comp * g.plane, plane.data(),
                        g.plane * sizeof(Real), hipMemcpyHostToDevice));
  }
  return PIC_OK;
}

// Particles [start, start + cnt) of the species in storage order.
template <typename Real>
int read_particles_t(pic_ctx* c, SpeciesHost& s, int64_t start, int64_t cnt, int32_t* cell,
                     double* off, double* delta, double* u1, double* u2, double* wc, double* w,
                     int64_t* id) {
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const int64_t n = cnt;
  const int nd = c->g.nd;
  if (n == 0) return PIC_OK;
  if (cell) {
    std::vector<uint32_t> pk(n);
    HIPCHK(c, hipMemcpy(pk.data(), static_cast<uint32_t*>(s.cell) + start, n * sizeof(uint32_t),
                        hipMemcpyDeviceToHost));
    for (int64_t p = 0; p < n; p++) {
      uint32_t v = pk[p];
      int ci[3] = {0, 0, 0};
      ci[0] = v & ((1u << c->g.bits[0]) - 1u);
      if (nd > 1) ci[1] = (v >> c->g.bits[0]) & ((1u << c->g.bits[1]) - 1u);
      if (nd > 2) ci[2] = v >> (c->g.bits[0] + c->g.bits[1]);
      for (int d = 0; d < 3; d++) cell[p * 3 + d] = ci[d];
    }
  }
  std::vector<Real> buf(n);
  // component `comp` of an n x `stride` host array from a device array
  auto get = [&](void* src, double* dst, int comp, int stride) -> int {
    HIPCHK(c, hipMemcpy(buf.data(), static_cast<Real*>(src) + start, n * sizeof(Real),
                        hipMemcpyDeviceToHost));
    for (int64_t p = 0; p < n; p++) dst[p * stride + comp] = (double)buf[p];
    return PIC_OK;
  };
  int rc;
  if (off) {
    for (int64_t p = 0; p < 3 * n; p++) off[p] = 0.0;
    for (int d = 0; d < nd; d++)
      if ((rc = get(s.off[d], off, d, 3))) return rc;
  }
  for (int a = 0; a < 3; a++) {
    if (u1 && (rc = get(s.u1[a], u1, a, 3))) return rc;
    if (s.d.kind == PIC_TWO_BODY) {
      if (u2 && (rc = get(s.u2[a], u2, a, 3))) return rc;
      if (delta && (rc = get(s.dl[a], delta, a, 3))) return rc;
    }
    for (int k = 0; k < s.nshell; k++) {  // multi-shell: 3 nshell values per particle
      if (u2 && (rc = get(s.su2[k][a], u2, 3 * k + a, 3 * s.nshell))) return rc;
      if (delta && (rc = get(s.sdl[k][a], delta, 3 * k + a, 3 * s.nshell))) return rc;
    }
  }
  if (wc) {
    if (s.has_wc) {
      if ((rc = get(s.wc, wc, 0, 1))) return rc;
    } else {
      for (int64_t p = 0; p < n; p++) wc[p] = s.d.omega_c;
    }
  }
  if (w) {
    if (s.has_w) {
      if ((rc = get(s.w, w, 0, 1))) return rc;
    } else {
      for (int64_t p = 0; p < n; p++) w[p] = 1.0;
    }
  }
  if (id) {
    if (!s.ids) return fail(c, PIC_ESTATE, "ids need PIC_FLAG_TRACK_IDS");
    HIPCHK(c, hipMemcpy(id, s.ids + start, n * sizeof(int64_t), hipMemcpyDeviceToHost));
  }
  return PIC_OK;
}

template <typename Real>
int rho_t(pic_ctx* c, double* rho) {
  deposit_rho<Real>(c, c->rho0);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const GridInfo& g = c->g;
  std::vector<double> plane(g.plane);
  HIPCHK(c, hipMemcpy(plane.data(), c->rho0, g.plane * sizeof(double), hipMemcpyDeviceToHost));
  for (int k = 0; k < g.n[2]; k++)
    for (int j = 0; j < g.n[1]; j++)
      for (int i = 0; i < g.n[0]; i++)
        rho[i + (int64_t)g.n[0] * (j + (int64_t)g.n[1] * k)] = plane[g.origin + i + j * g.sy + k * g.sz];
  return PIC_OK;
}

}  // namespace

// A fixed finite a_c given with omega_c fixes the bond's Coulomb constant
// (Sec. 2 / Sec. 3.1), so the ions of such a species share one omega_c;
// per-particle omega_c needs a derived a_c or the harmonic bond.
static bool own_omega_allowed(const SpeciesHost& s) {
  return s.d.kind != PIC_TWO_BODY || s.ac_derived || std::isinf(s.a_c);
}
static const char* const omega_fixed_msg =
    "per-particle omega_c needs a_c = 0 (derived per ion) or a_c = +inf (harmonic)";

// allocate the optional per-particle arrays on the first load that brings them
// After a sort: list, per colour, the tiles that hold particles (one small
// kernel and a read-back of the 8 counts, once per sort); when fewer than
// half of the tiles are occupied (a few ions in a large box, a crystal in
// part of it), the tiled launches visit only those, else every tile.
int update_occupancy(pic_ctx* c) {
  c->tg.occ = nullptr;
  if (!c->tiled || c->sp.empty() || c->sp.size() > (size_t)pic::kOccSpecies) return PIC_OK;
  const int64_t per_colour = (int64_t)c->tg.nc[0] * c->tg.nc[1] * c->tg.nc[2];
  const int64_t ntile = (int64_t)c->tg.nt[0] * c->tg.nt[1] * c->tg.nt[2];
  if (!c->occ) {
    c->occ = static_cast<uint32_t*>(dev_alloc(c, (size_t)(8 + 8 * per_colour) * 4));
    if (!c->occ) return fail(c, PIC_ENOMEM, "device allocation failed (occupied tiles)");
  }
  const uint32_t* offs[pic::kOccSpecies] = {};
  for (size_t s = 0; s < c->sp.size(); s++) offs[s] = c->sp[s]->sort.tile_off;
  hipError_t e =
      pic::launch_occupied_tiles(c->tg, offs, (int)c->sp.size(), c->occ, c->stream);
  if (e != hipSuccess) return fail(c, PIC_EHIP, std::string("occupied tiles: ") + hipGetErrorString(e));
  uint32_t n[8];
  HIPCHK(c, hipMemcpyAsync(n, c->occ, sizeof(n), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  int64_t busy = 0;
  for (int k = 0; k < 8; k++) busy += n[k];
  if (2 * busy >= ntile) return PIC_OK;
  for (int k = 0; k < 8; k++) c->tg.occ_n[k] = n[k];
  c->tg.occ = c->occ;
  return PIC_OK;
}

int prepare_optional(pic_ctx* c, SpeciesHost& s, bool want_wc, bool want_w) {
  size_t rs = c->rsize, cap = (size_t)s.cap;
  pic::AllocFn af = [c](size_t b) { return dev_alloc(c, b); };
  if (want_wc && !s.wc) {
    if (s.n > 0) return fail(c, PIC_ESTATE, "per-particle omega_c must come with the first load");
    if (!(s.wc = dev_alloc(c, cap * rs))) return fail(c, PIC_ENOMEM, "device allocation failed");
    if (pic::sort_add_attr(s.sort, &s.wc, rs, af))
      return fail(c, PIC_ENOMEM, "device allocation failed");
    s.has_wc = true;
  }
  if (want_w && !s.w) {
    if (s.n > 0) return fail(c, PIC_ESTATE, "per-particle weight must come with the first load");
    if (!(s.w = dev_alloc(c, cap * rs))) return fail(c, PIC_ENOMEM, "device allocation failed");
    if (pic::sort_add_attr(s.sort, &s.w, rs, af))
      return fail(c, PIC_ENOMEM, "device allocation failed");
    s.has_w = true;
  }
  return PIC_OK;
}

void harvest_pending_counts(pic_ctx* c) { harvest_counts(c); }

// ================================================================ C ABI

extern "C" {

const char* pic_version(void) { return "libpic 0.1 (gfx950)"; }

const char* pic_last_error(const pic_ctx* ctx) {
  return ctx ? ctx->error.c_str() : g_create_error.c_str();
}

int pic_create(const pic_config* cfg, const pic_allocator* alloc, void* hip_stream,
               pic_ctx** out) {
  if (!cfg || !out) return fail(nullptr, PIC_EINVAL, "null argument");
  *out = nullptr;
  if (cfg->ndim < 1 || cfg->ndim > 3) return fail(nullptr, PIC_EINVAL, "ndim must be 1, 2 or 3");
  if (cfg->precision != 32 && cfg->precision != 64)
    return fail(nullptr, PIC_EINVAL, "precision must be 32 or 64");
  if (!(cfg->dt > 0)) return fail(nullptr, PIC_EINVAL, "dt must be positive");
  double inv2 = 0.0;
  int bits = 0;
  for (int d = 0; d < cfg->ndim; d++) {
    if (cfg->n[d] < 1 || !(cfg->dx[d] > 0)) return fail(nullptr, PIC_EINVAL, "bad grid size");
    inv2 += 1.0 / (cfg->dx[d] * cfg->dx[d]);
    bits += ceil_log2(cfg->n[d]);
    bool pl = cfg->bc_lo[d] == PIC_BC_PERIODIC, ph = cfg->bc_hi[d] == PIC_BC_PERIODIC;
    if (pl != ph) return fail(nullptr, PIC_EINVAL, "periodic faces come in pairs");
    if (cfg->bc_hi[d] == PIC_BC_LASER || (d > 0 && cfg->bc_lo[d] == PIC_BC_LASER))
      return fail(nullptr, PIC_EINVAL, "the laser enters through x-min only");
    if (d == 0 && cfg->laser.angle != 0.0 && (cfg->ndim < 2 || cfg->laser.waist > 0.0))
      return fail(nullptr, PIC_EINVAL, "an oblique laser is a plane wave in 2D or 3D");
    if (pl && cfg->n[d] < 2 * pic::kGuard)
      return fail(nullptr, PIC_EINVAL, "periodic dimensions need at least 6 cells");
    if (!pl && cfg->pad < 3) return fail(nullptr, PIC_EINVAL, "pad must be >= 3 with open faces");
    if (!pl && cfg->n[d] < 2 * cfg->pad + 1)
      return fail(nullptr, PIC_EINVAL, "grid too small for the particle walls");
  }
  if (cfg->laser.n_env < 0 || cfg->laser.n_env > PIC_MAX_ENV)
    return fail(nullptr, PIC_EINVAL, "n_env must be in [0, PIC_MAX_ENV]");
  if (bits > 31) return fail(nullptr, PIC_EINVAL, "grid too large for the packed cell index");
  {
    int64_t plane = 1;
    for (int d = 0; d < cfg->ndim; d++) plane *= cfg->n[d] + 2 * pic::kGuard;
    if (plane >= (int64_t(1) << 31))
      return fail(nullptr, PIC_EINVAL, "field plane exceeds 2^31 values (32-bit indexing)");
  }
  if (!(cfg->dt * std::sqrt(inv2) < 1.0))
    return fail(nullptr, PIC_EINVAL, "time step violates the CFL limit");
  if (!alloc || !alloc->alloc || !alloc->free)
    return fail(nullptr, PIC_EINVAL, "an allocator with alloc and free is required");

  pic_ctx* c = new pic_ctx();
  c->cfg = *cfg;
  c->alloc = *alloc;
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return fail(nullptr, PIC_EHIP, "hipGetDevice failed");
  }
  c->prec = cfg->precision;
  c->rsize = cfg->precision == 32 ? 4 : 8;
  GridInfo& g = c->g;
  g.nd = cfg->ndim;
  g.plane = 1;
  g.pad = cfg->pad;
  for (int d = 0; d < 3; d++) {
    bool r = d < g.nd;
    g.n[d] = r ? (int)cfg->n[d] : 1;
    g.g[d] = r ? pic::kGuard : 0;
    g.st[d] = g.n[d] + 2 * g.g[d];
    g.periodic[d] = r ? (is_periodic(*cfg, d) ? 1 : 0) : 1;
    g.bits[d] = r ? ceil_log2(cfg->n[d]) : 0;
    g.dx[d] = r ? cfg->dx[d] : 1.0;
    g.plane *= g.st[d];
  }
  g.dt = cfg->dt;
  g.sy = g.st[0];
  g.sz = (int64_t)g.st[0] * g.st[1];
  g.origin = g.g[0] + g.g[1] * g.sy + g.g[2] * g.sz;
  // tiles
  // default tiles: in 3D FP32 an 8x8x6 tile lets two workgroups share a CU
  // (LDS under 80 KB); FP64 fields need the larger 8^3 tile's one per CU
  const int def3f[3] = {8, 8, 6}, def3d[3] = {8, 8, 8};
  const int def2[3] = {12, 12, 1}, def1[3] = {256, 1, 1};
  const int* def3 = cfg->precision == 32 ? def3f : def3d;
  const int* def = g.nd == 3 ? def3 : (g.nd == 2 ? def2 : def1);
  for (int d = 0; d < 3; d++) {
    int t = d < g.nd ? (cfg->tile[d] > 0 ? cfg->tile[d] : def[d]) : 1;
    if (d < g.nd) t = std::min(t, g.n[d]);
    c->tile[d] = std::max(t, 1);
    c->ntiles[d] = (g.n[d] + c->tile[d] - 1) / c->tile[d];
  }
  c->sort_every = cfg->sort_every > 0 ? cfg->sort_every : 0;
  c->tg = pic::make_tile_geom(g, c->tile, c->ntiles, c->rsize);
  c->tiled = !(cfg->flags & PIC_FLAG_GLOBAL_KERNEL) && pic::tiled_supported(g, c->tg, c->rsize);

  size_t rs = c->rsize;
  c->yee_fused = g.nd <= 2;  // 3D keeps the three streaming passes
  c->fields = dev_alloc(c, 6 * g.plane * rs);
  c->jfield = dev_alloc(c, 3 * g.plane * rs);
  c->fields_alt = c->yee_fused ? dev_alloc(c, 6 * g.plane * rs) : nullptr;
  c->err = static_cast<uint32_t*>(dev_alloc(c, 256));
  c->load_err = static_cast<uint32_t*>(dev_alloc(c, 256));
  c->nslow = static_cast<uint32_t*>(dev_alloc(c, 256));
  c->nfar = static_cast<uint32_t*>(dev_alloc(c, 256));
  c->partials = static_cast<double*>(dev_alloc(c, 8 * pic::reduce_blocks() * sizeof(double)));
  c->dout = static_cast<double*>(dev_alloc(c, 32 * sizeof(double)));
  c->rho0 = static_cast<double*>(dev_alloc(c, g.plane * sizeof(double)));
  c->rho1 = static_cast<double*>(dev_alloc(c, g.plane * sizeof(double)));
  if (!c->fields || !c->jfield || (c->yee_fused && !c->fields_alt) || !c->err || !c->load_err || !c->nslow || !c->nfar || !c->partials || !c->dout || !c->rho0 || !c->rho1) {
    dev_free_all(c);
    delete c;
    return fail(nullptr, PIC_ENOMEM, "device allocation failed");
  }
  for (int d = 0; d < g.nd; d++) {
    if (g.periodic[d]) continue;
    int a_dim = d == 0 ? 1 : 0, b_dim = d == 2 ? 1 : 2;
    size_t np = (size_t)g.n[a_dim] * g.n[b_dim];
    for (int t = 0; t < 2; t++) {
      c->mur_b[d][t] = dev_alloc(c, np * rs);
      c->mur_e[d][t] = dev_alloc(c, np * rs);
      if (c->yee_fused) c->mur_b_alt[d][t] = dev_alloc(c, np * rs);
      if (!c->mur_b[d][t] || !c->mur_e[d][t] || (c->yee_fused && !c->mur_b_alt[d][t])) {
        dev_free_all(c);
        delete c;
        return fail(nullptr, PIC_ENOMEM, "device allocation failed");
      }
    }
  }
  hipError_t e = hipMemsetAsync(c->fields, 0, 6 * g.plane * rs, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->jfield, 0, 3 * g.plane * rs, c->stream);
  if (e == hipSuccess && c->fields_alt)
    e = hipMemsetAsync(c->fields_alt, 0, 6 * g.plane * rs, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->err, 0, 256, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->nslow, 0, 256, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->nfar, 0, 256, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->dout, 0, 32 * sizeof(double), c->stream);
  for (int d = 0; d < g.nd && e == hipSuccess; d++) {
    if (g.periodic[d]) continue;
    int a_dim = d == 0 ? 1 : 0, b_dim = d == 2 ? 1 : 2;
    size_t np = (size_t)g.n[a_dim] * g.n[b_dim];
    for (int t = 0; t < 2 && e == hipSuccess; t++) {
      e = hipMemsetAsync(c->mur_b[d][t], 0, np * rs, c->stream);
      if (e == hipSuccess) e = hipMemsetAsync(c->mur_e[d][t], 0, np * rs, c->stream);
      if (e == hipSuccess && c->mur_b_alt[d][t])
        e = hipMemsetAsync(c->mur_b_alt[d][t], 0, np * rs, c->stream);
    }
  }
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->host_counts, 2 * 128 * sizeof(uint32_t));
  for (int t = 0; t < 2 && e == hipSuccess; t++) e = hipEventCreate(&c->ev_counts[t]);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    std::string msg = std::string("HIP: ") + hipGetErrorString(e);
    release_host(c);
    dev_free_all(c);
    delete c;
    return fail(nullptr, PIC_EHIP, msg);
  }
  *out = c;
  return PIC_OK;
}

int pic_add_species(pic_ctx* c, const pic_species_desc* d, int32_t* sid) {
  if (!c || !d || !sid) return fail(c, PIC_EINVAL, "null argument");
  c->version++;  // a gradient run started before this can no longer be reversed
  if (d->kind != PIC_POINT && d->kind != PIC_TWO_BODY) return fail(c, PIC_EINVAL, "bad kind");
  if ((int)c->sp.size() >= kMaxSpecies) return fail(c, PIC_EINVAL, "too many species");
  if (d->capacity < 0 || d->capacity >= (int64_t(1) << 31))
    return fail(c, PIC_EINVAL, "capacity must be below 2^31");
  if (!(d->m1 > 0) || d->q1 == 0.0) return fail(c, PIC_EINVAL, "bad charge or mass");
  auto holder = std::make_unique<SpeciesHost>();
  SpeciesHost& s = *holder;
  s.d = *d;
  s.cap = std::max<int64_t>(d->capacity, 1);
  const bool two = d->kind == PIC_TWO_BODY;
  if (two) {
    if (!(d->m2 > 0) || d->q2 == 0.0) return fail(c, PIC_EINVAL, "bad bound-electron charge/mass");
    if (!(d->omega_c > 0)) return fail(c, PIC_EINVAL, "omega_c must be positive");
    if (std::isnan(d->a_c) || d->a_c < 0)
      return fail(c, PIC_EINVAL, "a_c must be 0 (derived), positive or +inf");
    double mr = d->m1 * d->m2 / (d->m1 + d->m2);
    if (std::isinf(d->a_c))
      s.a_c = std::numeric_limits<double>::infinity();
    else if (d->a_c > 0)
      s.a_c = d->a_c;
    else {
      // Sec. 3.1: w_c^2 = |q1 q2| (Coulomb constant) / (m_r a_c^3), the
      // Coulomb constant being re_norm in these units
      if (!(c->cfg.re_norm > 0)) return fail(c, PIC_EINVAL, "a_c = 0 needs re_norm > 0");
      s.a_c = std::cbrt(std::fabs(d->q1 * d->q2) * c->cfg.re_norm / (mr * d->omega_c * d->omega_c));
      s.ac_derived = true;  // and each ion's own from its own omega_c
    }
  }
  size_t rs = c->rsize, n = (size_t)s.cap;
  s.cell = dev_alloc(c, n * 4);
  bool ok = s.cell != nullptr;
  for (int a = 0; a < c->g.nd; a++) ok = ok && (s.off[a] = dev_alloc(c, n * rs));
  for (int a = 0; a < 3; a++) {
    ok = ok && (s.u1[a] = dev_alloc(c, n * rs));
    if (two) {
      ok = ok && (s.u2[a] = dev_alloc(c, n * rs));
      ok = ok && (s.dl[a] = dev_alloc(c, n * rs));
    }
  }
  if (c->cfg.flags & PIC_FLAG_TRACK_IDS)
    ok = ok && (s.ids = static_cast<int64_t*>(dev_alloc(c, n * sizeof(int64_t))));
  if (c->tiled) ok = ok && (s.outside = static_cast<uint32_t*>(dev_alloc(c, n * 4)));
  if (!ok) return fail(c, PIC_ENOMEM, "device allocation failed");
  pic::AllocFn af = [c](size_t b) { return dev_alloc(c, b); };
  int rc = pic::sort_alloc(c->g, c->ntiles, s.cap, af, s.sort);
  rc = rc || pic::sort_add_attr(s.sort, &s.cell, 4, af);
  for (int a = 0; a < c->g.nd && !rc; a++) rc = pic::sort_add_attr(s.sort, &s.off[a], rs, af);
  for (int a = 0; a < 3 && !rc; a++) {
    rc = pic::sort_add_attr(s.sort, &s.u1[a], rs, af);
    if (two && !rc) rc = pic::sort_add_attr(s.sort, &s.u2[a], rs, af);
    if (two && !rc) rc = pic::sort_add_attr(s.sort, &s.dl[a], rs, af);
  }
  if (s.ids && !rc) rc = pic::sort_add_attr(s.sort, reinterpret_cast<void**>(&s.ids), 8, af);
  if (rc) return fail(c, PIC_ENOMEM, "device allocation failed (sort buffers)");
  c->sp.push_back(std::move(holder));
  *sid = (int32_t)(c->sp.size() - 1);
  return PIC_OK;
}

int pic_add_multishell(pic_ctx* c, const pic_species_desc* d, int32_t nshell,
                       const double* shell_q, const double* shell_m, const double* shell_omega,
                       const double* shell_ac, int32_t* sid) {
  if (!c || !d || !sid || !shell_q || !shell_m || !shell_omega || !shell_ac)
    return fail(c, PIC_EINVAL, "null argument");
  c->version++;
  if (d->kind != PIC_MULTI_SHELL) return fail(c, PIC_EINVAL, "bad kind (PIC_MULTI_SHELL expected)");
  if (nshell < 1 || nshell > pic::kMaxShell)
    return fail(c, PIC_EINVAL, "nshell must be 1 .. PIC_MAX_SHELL");
  if ((int)c->sp.size() >= kMaxSpecies) return fail(c, PIC_EINVAL, "too many species");
  if (d->capacity < 0 || d->capacity >= (int64_t(1) << 31))
    return fail(c, PIC_EINVAL, "capacity must be below 2^31");
  if (!(d->m1 > 0) || d->q1 == 0.0) return fail(c, PIC_EINVAL, "bad nucleus charge or mass");
  if (std::isnan(d->nu) || d->nu < 0) return fail(c, PIC_EINVAL, "nu must be >= 0");
  auto holder = std::make_unique<SpeciesHost>();
  SpeciesHost& s = *holder;
  s.d = *d;
  s.d.q2 = s.d.m2 = s.d.omega_c = s.d.a_c = s.d.nu_per_omega = 0.0;
  s.cap = std::max<int64_t>(d->capacity, 1);
  s.nshell = nshell;
  for (int k = 0; k < nshell; k++) {
    if (!(shell_m[k] > 0) || shell_q[k] == 0.0 || !std::isfinite(shell_q[k]))
      return fail(c, PIC_EINVAL, "bad cloud charge or mass");
    if (!(shell_omega[k] > 0)) return fail(c, PIC_EINVAL, "shell omega_c must be positive");
    if (std::isnan(shell_ac[k]) || shell_ac[k] < 0)
      return fail(c, PIC_EINVAL, "shell a_c must be 0 (derived), positive or +inf");
    s.sq[k] = shell_q[k];
    s.sm[k] = shell_m[k];
    s.sw[k] = shell_omega[k];
    if (shell_ac[k] > 0) {
      s.sa[k] = shell_ac[k];
    } else {
      // as for a two-body ion, with the nucleus-cloud pair's reduced mass
      if (!(c->cfg.re_norm > 0)) return fail(c, PIC_EINVAL, "a_c = 0 needs re_norm > 0");
      const double mr = d->m1 * shell_m[k] / (d->m1 + shell_m[k]);
      s.sa[k] = std::cbrt(std::fabs(d->q1 * shell_q[k]) * c->cfg.re_norm /
                          (mr * shell_omega[k] * shell_omega[k]));
    }
  }
  size_t rs = c->rsize, n = (size_t)s.cap;
  s.cell = dev_alloc(c, n * 4);
  bool ok = s.cell != nullptr;
  for (int a = 0; a < c->g.nd; a++) ok = ok && (s.off[a] = dev_alloc(c, n * rs));
  for (int a = 0; a < 3; a++) {
    ok = ok && (s.u1[a] = dev_alloc(c, n * rs));
    for (int k = 0; k < nshell; k++) {
      ok = ok && (s.sdl[k][a] = dev_alloc(c, n * rs));
      ok = ok && (s.su2[k][a] = dev_alloc(c, n * rs));
    }
  }
  if (c->cfg.flags & PIC_FLAG_TRACK_IDS)
    ok = ok && (s.ids = static_cast<int64_t*>(dev_alloc(c, n * sizeof(int64_t))));
  if (!ok) return fail(c, PIC_ENOMEM, "device allocation failed");
  pic::AllocFn af = [c](size_t b) { return dev_alloc(c, b); };
  int rc = pic::sort_alloc(c->g, c->ntiles, s.cap, af, s.sort);
  rc = rc || pic::sort_add_attr(s.sort, &s.cell, 4, af);
  for (int a = 0; a < c->g.nd && !rc; a++) rc = pic::sort_add_attr(s.sort, &s.off[a], rs, af);
  for (int a = 0; a < 3 && !rc; a++) {
    rc = pic::sort_add_attr(s.sort, &s.u1[a], rs, af);
    for (int k = 0; k < nshell && !rc; k++) {
      rc = pic::sort_add_attr(s.sort, &s.sdl[k][a], rs, af);
      if (!rc) rc = pic::sort_add_attr(s.sort, &s.su2[k][a], rs, af);
    }
  }
  if (s.ids && !rc) rc = pic::sort_add_attr(s.sort, reinterpret_cast<void**>(&s.ids), 8, af);
  if (rc) return fail(c, PIC_ENOMEM, "device allocation failed (sort buffers)");
  c->sp.push_back(std::move(holder));
  *sid = (int32_t)(c->sp.size() - 1);
  return PIC_OK;
}

int pic_load_particles(pic_ctx* c, int32_t sid, int64_t n, const double* x, const double* delta,
                       const double* u1, const double* u2, const double* omega_c,
                       const double* weight) {
  if (!c) return PIC_EINVAL;
  c->version++;  // a gradient run started before this can no longer be reversed
  if (sid < 0 || sid >= (int32_t)c->sp.size()) return fail(c, PIC_ESTATE, "unknown species");
  if (n < 0 || (n > 0 && (!x || !u1))) return fail(c, PIC_EINVAL, "null particle arrays");
  SpeciesHost& s = *c->sp[sid];
  if (s.n + n > s.cap) return fail(c, PIC_ENOMEM, "species capacity exceeded");
  if (n == 0) return PIC_OK;
  if (omega_c && !own_omega_allowed(s))
    return fail(c, PIC_EINVAL, omega_fixed_msg);
  if (s.d.kind == PIC_MULTI_SHELL && omega_c)
    return fail(c, PIC_EINVAL, "the bond frequencies of a multi-shell species are per shell");
  int rc = prepare_optional(c, s, omega_c != nullptr, weight != nullptr);
  if (rc) return rc;
  if (s.d.kind == PIC_MULTI_SHELL)
    return c->prec == 32 ? load_shells_t<float>(c, s, n, x, delta, u1, u2, weight)
                         : load_shells_t<double>(c, s, n, x, delta, u1, u2, weight);
  if (c->prec == 32) return load_particles_t<float>(c, s, n, x, delta, u1, u2, omega_c, weight);
  return load_particles_t<double>(c, s, n, x, delta, u1, u2, omega_c, weight);
}

int pic_load_particles_device(pic_ctx* c, int32_t sid, int64_t n, const double* x,
                              const double* delta, const double* u1, const double* u2,
                              const double* omega_c, const double* weight) {
  if (!c) return PIC_EINVAL;
  c->version++;  // a gradient run started before this can no longer be reversed
  if (sid < 0 || sid >= (int32_t)c->sp.size()) return fail(c, PIC_ESTATE, "unknown species");
  if (n < 0 || (n > 0 && (!x || !u1))) return fail(c, PIC_EINVAL, "null particle arrays");
  SpeciesHost& s = *c->sp[sid];
  if (s.n + n > s.cap) return fail(c, PIC_ENOMEM, "species capacity exceeded");
  if (n == 0) return PIC_OK;
  const bool shells = s.d.kind == PIC_MULTI_SHELL;
  if (shells && omega_c)
    return fail(c, PIC_EINVAL, "the bond frequencies of a multi-shell species are per shell");
  if (omega_c && !own_omega_allowed(s))
    return fail(c, PIC_EINVAL, omega_fixed_msg);
  int rc = prepare_optional(c, s, omega_c != nullptr, weight != nullptr);
  if (rc) return rc;
  HIPCHK(c, hipMemsetAsync(c->load_err, 0, 16, c->stream));
  if (shells) {
    pic::ShellLoad src{};
    src.x = x;
    src.delta = delta;
    src.u1 = u1;
    src.u2 = u2;
    src.w = weight;
    src.n = n;
    src.weight = s.d.weight;
    src.K = s.nshell;
    double M = s.d.m1;
    for (int k = 0; k < s.nshell; k++) M += s.sm[k];
    src.fm[0] = s.d.m1 / M;
    for (int k = 0; k < s.nshell; k++) src.fm[k + 1] = s.sm[k] / M;
    if (c->prec == 32)
      pic::launch_load_shells<float>(c->g, src, shell_dev<float>(s), s.n, s.ids, c->load_err,
                                     c->stream);
    else
      pic::launch_load_shells<double>(c->g, src, shell_dev<double>(s), s.n, s.ids, c->load_err,
                                      c->stream);
  } else {
    pic::LoadSrc src{x, delta, u1, u2, omega_c, weight, n};
    pic::LoadSplit sp{s.d.q1, s.d.m1, s.d.q2, s.d.m2, s.d.omega_c, s.d.weight};
    const bool two = s.d.kind == PIC_TWO_BODY;
    if (c->prec == 32)
      pic::launch_load<float>(c->g, src, species_dev<float>(s), s.n, s.ids, sp, two,
                              c->load_err, c->stream);
    else
      pic::launch_load<double>(c->g, src, species_dev<double>(s), s.n, s.ids, sp, two,
                               c->load_err, c->stream);
  }
  uint32_t lw[4] = {0, 0, 0, 0};
  HIPCHK(c, hipMemcpyAsync(lw, c->load_err, 16, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const uint32_t bad = lw[0];
  if (s.has_w) {  // bytes 8..15: bits of the largest |weight| of this load
    uint64_t bits = (uint64_t)lw[2] | ((uint64_t)lw[3] << 32);
    double wm;
    std::memcpy(&wm, &bits, sizeof(wm));
    s.max_w = std::max(s.max_w, wm);
  }
  if (bad & PIC_ERR_NAN) return fail(c, PIC_ENAN, "non-finite particle state");
  if (bad & PIC_ERR_RANGE) return fail(c, PIC_ERANGE, "particle outside the grid, walls or bond range");
  s.n += n;
  if (pic::sort_by_tile(c->g, c->tile, c->ntiles, s.sort, s.n, c->stream, true))
    return fail(c, PIC_EHIP, "tile sort failed");
  s.needs_sort = false;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PIC_OK;
}

int pic_load_fields(pic_ctx* c, const double* E, const double* B) {
  if (!c) return PIC_EINVAL;
  c->version++;  // a gradient run started before this can no longer be reversed
  return c->prec == 32 ? load_fields_t<float>(c, E, B) : load_fields_t<double>(c, E, B);
}

int pic_step(pic_ctx* c, int32_t nsteps) {
  if (!c || nsteps < 0) return c ? fail(c, PIC_EINVAL, "nsteps < 0") : PIC_EINVAL;
  c->version++;  // a gradient run started before this can no longer be reversed
  return c->prec == 32 ? step_t<float>(c, nsteps) : step_t<double>(c, nsteps);
}

int pic_diagnostics(pic_ctx* c, pic_diag* out) {
  if (!c || !out) return PIC_EINVAL;
  return c->prec == 32 ? diagnostics_t<float>(c, out) : diagnostics_t<double>(c, out);
}

int pic_read_fields(pic_ctx* c, double* E, double* B, double* J) {
  if (!c) return PIC_EINVAL;
  return c->prec == 32 ? read_fields_t<float>(c, E, B, J) : read_fields_t<double>(c, E, B, J);
}

int pic_count(pic_ctx* c, int32_t sid, int64_t* n) {
  if (!c || !n) return PIC_EINVAL;
  if (sid < 0 || sid >= (int32_t)c->sp.size()) return fail(c, PIC_ESTATE, "unknown species");
  *n = c->sp[sid]->n;
  return PIC_OK;
}

int pic_read_particles(pic_ctx* c, int32_t sid, int32_t* cell, double* offset, double* delta,
                       double* u1, double* u2, int64_t* id) {
  if (!c) return PIC_EINVAL;
  if (sid < 0 || sid >= (int32_t)c->sp.size()) return fail(c, PIC_ESTATE, "unknown species");
  SpeciesHost& s = *c->sp[sid];
  return c->prec == 32
             ? read_particles_t<float>(c, s, 0, s.n, cell, offset, delta, u1, u2, nullptr,
                                       nullptr, id)
             : read_particles_t<double>(c, s, 0, s.n, cell, offset, delta, u1, u2, nullptr,
                                        nullptr, id);
}

int pic_read_particles_range(pic_ctx* c, int32_t sid, int64_t start, int64_t count,
                             int32_t* cell, double* offset, double* delta, double* u1, double* u2,
                             double* omega_c, double* weight, int64_t* id) {
  if (!c) return PIC_EINVAL;
  if (sid < 0 || sid >= (int32_t)c->sp.size()) return fail(c, PIC_ESTATE, "unknown species");
  SpeciesHost& s = *c->sp[sid];
  if (start < 0 || count < 0 || start > s.n || count > s.n - start)
    return fail(c, PIC_EINVAL, "particle range outside the species");
  return c->prec == 32 ? read_particles_t<float>(c, s, start, count, cell, offset, delta, u1, u2,
                                                 omega_c, weight, id)
                       : read_particles_t<double>(c, s, start, count, cell, offset, delta, u1,
                                                  u2, omega_c, weight, id);
}

int pic_rho(pic_ctx* c, double* rho) {
  if (!c || !rho) return PIC_EINVAL;
  return c->prec == 32 ? rho_t<float>(c, rho) : rho_t<double>(c, rho);
}

int pic_set_probes(pic_ctx* c, int32_t nprobe, const int32_t* comp, const int64_t* ijk) {
  if (!c || nprobe < 0 || (nprobe > 0 && (!comp || !ijk))) return PIC_EINVAL;
  c->version++;  // a gradient run started before this can no longer be reversed
  if (nprobe > 0 && c->cfg.max_probe_steps <= 0)
    return fail(c, PIC_EINVAL, "max_probe_steps must be positive to record probes");
  if (nprobe > c->nprobe) {
    c->probe_comp = static_cast<int*>(dev_alloc(c, nprobe * sizeof(int)));
    c->probe_idx = static_cast<int64_t*>(dev_alloc(c, nprobe * sizeof(int64_t)));
    c->probe_buf = dev_alloc(c, (size_t)nprobe * c->cfg.max_probe_steps * c->rsize);
    if (!c->probe_comp || !c->probe_idx || !c->probe_buf)
      return fail(c, PIC_ENOMEM, "device allocation failed");
  }
  std::vector<int> hc(nprobe);
  std::vector<int64_t> hi(nprobe);
  for (int p = 0; p < nprobe; p++) {
    if (comp[p] < 0 || comp[p] > 5) return fail(c, PIC_EINVAL, "probe component must be 0..5");
    int64_t ix[3];
    for (int d = 0; d < 3; d++) {
      ix[d] = ijk[3 * p + d];
      if (ix[d] < 0 || ix[d] >= c->g.n[d]) return fail(c, PIC_EINVAL, "probe outside the grid");
    }
    hc[p] = comp[p];
    hi[p] = c->g.origin + ix[0] + ix[1] * c->g.sy + ix[2] * c->g.sz;
  }
  if (nprobe > 0) {
    HIPCHK(c, hipMemcpy(c->probe_comp, hc.data(), nprobe * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->probe_idx, hi.data(), nprobe * sizeof(int64_t), hipMemcpyHostToDevice));
  }
  c->nprobe = nprobe;
  c->probe_rec = 0;
  return PIC_OK;
}

int pic_read_probes(pic_ctx* c, double* out, int64_t* nrec) {
  if (!c) return PIC_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (nrec) *nrec = c->probe_rec;
  if (!out || c->nprobe == 0 || c->probe_rec == 0) return PIC_OK;
  size_t total = (size_t)c->nprobe * c->cfg.max_probe_steps;
  if (c->prec == 32) {
    std::vector<float> b(total);
    HIPCHK(c, hipMemcpy(b.data(), c->probe_buf, total * 4, hipMemcpyDeviceToHost));
    for (int p = 0; p < c->nprobe; p++)
      for (int64_t t = 0; t < c->probe_rec; t++)
        out[p * c->probe_rec + t] = b[(size_t)p * c->cfg.max_probe_steps + t];
  } else {
    std::vector<double> b(total);
    HIPCHK(c, hipMemcpy(b.data(), c->probe_buf, total * 8, hipMemcpyDeviceToHost));
    for (int p = 0; p < c->nprobe; p++)
      for (int64_t t = 0; t < c->probe_rec; t++)
        out[p * c->probe_rec + t] = b[(size_t)p * c->cfg.max_probe_steps + t];
  }
  return PIC_OK;
}

int pic_timing(pic_ctx* c, int32_t species_id, double* total_ms, int64_t* launches,
               int32_t reset) {
  if (!c) return PIC_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double tot = 0.0;
  int64_t cnt = 0;
  for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
    if (species_id >= 0 && c->ev_species[i / 2] != species_id) continue;
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
    tot += ms;
    cnt++;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = cnt;
  if (reset) c->ev_used = 0;
  return PIC_OK;
}

void pic_destroy(pic_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  grad_release(c);
  release_host(c);
  dev_free_all(c);
  delete c;
}

}  // extern "C"
