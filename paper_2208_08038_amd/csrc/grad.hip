// grad.hip -- gradient run: reverse-mode (adjoint) differentiation of the
// step with checkpointing.
//
// pic_grad_forward advances the system as pic_step does (no tile sorts in
// between, so the storage order of the particles stays fixed) and keeps a
// snapshot of the whole state every K steps.  pic_grad_backward walks the
// checkpoint segments from the last to the first: it restores the
// segment's checkpoint, re-runs its steps keeping the state at the start
// of each, then reverses them one by one.  Reversing step n applies, in
// reverse order, the transpose of every operation of the step:
//   probe recording -> B half step -> Mur E (high faces) -> E guard fill
//   -> E full step (gives the adjoint current lJ = -dt lE) -> high-face E
//   save -> Mur B (low faces; the laser's spline coefficients get their
//   gradient here) -> B guard fill -> B half step -> J guard fold ->
//   particle cycle of every species (adjoint kernel) -> E, B guard fill.
// What the reverse sweep leaves in the adjoint arrays is the gradient of
// the recorded probes' cotangent with respect to the state at the start of
// the run; the parameter gradients are accumulated on the way.
#include <cstring>

#include "adjoint.h"
#include "ctx.h"

namespace {

size_t up256(size_t b) { return (b + 255) & ~size_t(255); }

// Byte offsets of the pieces of a state snapshot.
struct SnapLayout {
  struct Sp {
    size_t cell, off[3], dl[3], u1[3], u2[3];
  };
  std::vector<Sp> sp;
  size_t fields = 0;        // E, B: 6 planes
  size_t mur[3][2] = {};    // Mur history of the low faces
  size_t bytes = 0;
};

SnapLayout snap_layout(const pic_ctx* c) {
  SnapLayout L;
  const size_t rs = c->rsize;
  size_t at = 0;
  for (auto& s : c->sp) {
    SnapLayout::Sp q{};
    const size_t n = (size_t)s->n;
    q.cell = at;
    at += up256(n * 4);
    for (int d = 0; d < 3; d++) {
      q.off[d] = at;
      if (d < c->g.nd) at += up256(n * rs);
    }
    for (int a = 0; a < 3; a++) {
      q.u1[a] = at;
      at += up256(n * rs);
    }
    if (s->d.kind == PIC_TWO_BODY)
      for (int a = 0; a < 3; a++) {
        q.u2[a] = at;
        at += up256(n * rs);
        q.dl[a] = at;
        at += up256(n * rs);
      }
    L.sp.push_back(q);
  }
  L.fields = at;
  at += up256(6 * (size_t)c->g.plane * rs);
  for (int d = 0; d < c->g.nd; d++) {
    if (c->g.periodic[d]) continue;
    int a_dim = d == 0 ? 1 : 0, b_dim = d == 2 ? 1 : 2;
    size_t np = (size_t)c->g.n[a_dim] * c->g.n[b_dim];
    for (int t = 0; t < 2; t++) {
      L.mur[d][t] = at;
      at += up256(np * rs);
    }
  }
  L.bytes = at;
  return L;
}

size_t face_bytes(const pic_ctx* c, int d) {
  int a_dim = d == 0 ? 1 : 0, b_dim = d == 2 ? 1 : 2;
  return (size_t)c->g.n[a_dim] * c->g.n[b_dim] * c->rsize;
}

}  // namespace

// slot of the gradient buffer that counts ions the reverse cycle skipped
// because their bodies were far apart (2 * 62 species + 64 coefficients < 255)
constexpr int kFarSlot = 255;

struct GradState {
  int64_t nsteps = 0, step0 = 0, rec0 = 0;
  int K = 0;
  bool ready = false;
  SnapLayout lay;
  std::vector<int64_t> sp_n;      // species sizes of the run
  std::vector<void*> ck;          // checkpoints (state at steps 0, K, 2K, ...)
  std::vector<int64_t> ck_step;
  std::vector<void*> slot;        // states at the start of each step of a segment
  void* final_state = nullptr;    // state at the end of the forward run
  int64_t final_step = 0;
  void* lam_fields = nullptr;     // adjoint E, B, J (9 planes)
  void* lam_mur_b[3][2] = {};     // adjoint of the Mur history of the low faces
  void* lam_mur_e[3][2] = {};     // adjoint of the saved high-face E (within a step)
  std::vector<void*> lam_sp;      // per species: adjoint offsets, delta, u1, u2
  double* dgrad = nullptr;        // [2 * nspecies + 64]: d omega_c, d nu, d env; [kFarSlot]
  double* dprobe = nullptr;
  size_t dprobe_cap = 0;
  // buffers are kept for the next run when the state has the same size
  size_t alloc_bytes = 0;
  uint64_t version = 0;           // context version at the end of the forward run
};

void grad_release(pic_ctx* c) {
  delete c->grad;  // device memory belongs to the context's allocation list
  c->grad = nullptr;
}

namespace {

// The pieces of one snapshot copy, moved by one kernel launch: piece
// blockIdx.y, 16-byte chunks over a grid-stride loop (a piece's size is a
// multiple of 4 bytes; the last chunk may be shorter).
constexpr int kMaxPieces = 48;
struct CopyList {
  const uint32_t* src[kMaxPieces];
  uint32_t* dst[kMaxPieces];
  int64_t words[kMaxPieces];
  int n;
};

__global__ void __launch_bounds__(256) k_copy_list(CopyList L) {
  const int k = blockIdx.y;
  const uint32_t* src = L.src[k];
  uint32_t* dst = L.dst[k];
  const int64_t nw = L.words[k];
  const int64_t nq = (nw + 3) / 4;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += stride) {
    const int64_t w = 4 * q;
    if (w + 4 <= nw) {
      *reinterpret_cast<uint4*>(dst + w) = *reinterpret_cast<const uint4*>(src + w);
    } else {
      for (int64_t i = w; i < nw; i++) dst[i] = src[i];
    }
  }
}

// Device-to-device copies between the live state and a snapshot: one
// kernel for every piece whose addresses are 16-byte aligned and size a
// multiple of 4 bytes, hipMemcpyAsync for any other.
int snap_copy(pic_ctx* c, void* buf, bool save) {
  const SnapLayout& L = c->grad->lay;
  char* b = static_cast<char*>(buf);
  const size_t rs = c->rsize;
  CopyList list{};
  auto cp = [&](void* live, size_t at, size_t bytes) -> int {
    void* dst = save ? (void*)(b + at) : live;
    const void* src = save ? (const void*)live : (const void*)(b + at);
    const bool fits = list.n < kMaxPieces && bytes % 4 == 0 &&
                      (reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) % 16 == 0;
    if (fits) {
      list.src[list.n] = static_cast<const uint32_t*>(src);
      list.dst[list.n] = static_cast<uint32_t*>(dst);
      list.words[list.n] = (int64_t)(bytes / 4);
      list.n++;
    } else {
      HIPCHK(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->stream));
    }
    return PIC_OK;
  };
  int rc;
  for (size_t si = 0; si < c->sp.size(); si++) {
    SpeciesHost& s = *c->sp[si];
    const SnapLayout::Sp& q = L.sp[si];
    const size_t n = (size_t)s.n;
    if (n == 0) continue;
    if ((rc = cp(s.cell, q.cell, n * 4))) return rc;
    for (int d = 0; d < c->g.nd; d++)
      if ((rc = cp(s.off[d], q.off[d], n * rs))) return rc;
    for (int a = 0; a < 3; a++) {
      if ((rc = cp(s.u1[a], q.u1[a], n * rs))) return rc;
      if (s.d.kind == PIC_TWO_BODY) {
        if ((rc = cp(s.u2[a], q.u2[a], n * rs))) return rc;
        if ((rc = cp(s.dl[a], q.dl[a], n * rs))) return rc;
      }
    }
  }
  if ((rc = cp(c->fields, L.fields, 6 * (size_t)c->g.plane * rs))) return rc;
  for (int d = 0; d < c->g.nd; d++) {
    if (c->g.periodic[d]) continue;
    for (int t = 0; t < 2; t++)
      if ((rc = cp(c->mur_b[d][t], L.mur[d][t], face_bytes(c, d)))) return rc;
  }
  if (list.n > 0) {
    hipLaunchKernelGGL(k_copy_list, dim3(256, list.n), 256, 0, c->stream, list);
    HIPCHK(c, hipGetLastError());
  }
  return PIC_OK;
}

struct SaveArg {
  void* buf;
  int rc;
};

void save_cb(pic_ctx* c, void* arg) {
  auto* a = static_cast<SaveArg*>(arg);
  if (a->rc == PIC_OK) a->rc = snap_copy(c, a->buf, true);
}

void* grad_alloc(pic_ctx* c, size_t bytes) { return dev_alloc(c, bytes); }

// Make sure the run's buffers exist (same-sized buffers are reused).
int grad_buffers(pic_ctx* c, int64_t nsteps, int K) {
  GradState& G = *c->grad;
  const SnapLayout L = snap_layout(c);
  std::vector<int64_t> sizes;
  for (auto& s : c->sp) sizes.push_back(s->n);
  if (L.bytes != G.alloc_bytes || sizes != G.sp_n) {
    // a different state size: release the previous run's snapshots and
    // particle adjoints (the field-sized buffers keep their size)
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (void* p : G.ck) dev_release(c, p);
    for (void* p : G.slot) dev_release(c, p);
    for (void* p : G.lam_sp) dev_release(c, p);
    dev_release(c, G.final_state);
    G.ck.clear();
    G.slot.clear();
    G.lam_sp.clear();
    G.final_state = nullptr;
    G.alloc_bytes = L.bytes;
  }
  G.lay = L;
  G.sp_n = sizes;
  const size_t nck = (size_t)((nsteps + K - 1) / K);
  while (G.ck.size() < nck) {
    void* p = grad_alloc(c, L.bytes);
    if (!p) return fail(c, PIC_ENOMEM, "device allocation of a checkpoint failed");
    G.ck.push_back(p);
  }
  while (G.slot.size() < (size_t)K) {
    void* p = grad_alloc(c, L.bytes);
    if (!p) return fail(c, PIC_ENOMEM, "device allocation of a step state failed");
    G.slot.push_back(p);
  }
  if (!G.final_state && !(G.final_state = grad_alloc(c, L.bytes)))
    return fail(c, PIC_ENOMEM, "device allocation failed");
  const size_t rs = c->rsize;
  if (!G.lam_fields && !(G.lam_fields = grad_alloc(c, 9 * (size_t)c->g.plane * rs)))
    return fail(c, PIC_ENOMEM, "device allocation failed");
  for (int d = 0; d < c->g.nd; d++) {
    if (c->g.periodic[d]) continue;
    for (int t = 0; t < 2; t++) {
      if (!G.lam_mur_b[d][t] && !(G.lam_mur_b[d][t] = grad_alloc(c, face_bytes(c, d))))
        return fail(c, PIC_ENOMEM, "device allocation failed");
      if (!G.lam_mur_e[d][t] && !(G.lam_mur_e[d][t] = grad_alloc(c, face_bytes(c, d))))
        return fail(c, PIC_ENOMEM, "device allocation failed");
    }
  }
  if (G.lam_sp.size() != c->sp.size()) {
    G.lam_sp.clear();
    for (auto& s : c->sp) {
      void* p = grad_alloc(c, (size_t)std::max<int64_t>(s->n, 1) * 12 * rs + 256 * 12);
      if (!p) return fail(c, PIC_ENOMEM, "device allocation failed");
      G.lam_sp.push_back(p);
    }
  }
  if (!G.dgrad && !(G.dgrad = static_cast<double*>(grad_alloc(c, 256 * sizeof(double)))))
    return fail(c, PIC_ENOMEM, "device allocation failed");
  return PIC_OK;
}

// Adjoint particle arrays of species si: 12 planes of n values (offsets
// 0..2, delta 3..5, u1 6..8, u2 9..11), each 256-byte aligned.
template <typename Real>
pic::AdjState<Real> lam_state(pic_ctx* c, size_t si) {
  pic::AdjState<Real> a{};
  const size_t n = (size_t)c->sp[si]->n;
  const size_t pitch = up256(std::max<size_t>(n, 1) * sizeof(Real));
  char* b = static_cast<char*>(c->grad->lam_sp[si]);
  for (int q = 0; q < 3; q++) {
    a.off[q] = reinterpret_cast<Real*>(b + (0 + q) * pitch);
    a.dl[q] = reinterpret_cast<Real*>(b + (3 + q) * pitch);
    a.u1[q] = reinterpret_cast<Real*>(b + (6 + q) * pitch);
    a.u2[q] = reinterpret_cast<Real*>(b + (9 + q) * pitch);
  }
  a.n = (int64_t)n;
  return a;
}

// The stored state of species si in a snapshot, with the species' own
// per-particle omega_c and weight.
template <typename Real>
pic::AdjState<Real> snap_state(pic_ctx* c, void* buf, size_t si) {
  const SpeciesHost& s = *c->sp[si];
  const SnapLayout::Sp& q = c->grad->lay.sp[si];
  char* b = static_cast<char*>(buf);
  pic::AdjState<Real> a = species_dev<Real>(s);
  a.cell = reinterpret_cast<uint32_t*>(b + q.cell);
  for (int d = 0; d < 3; d++) a.off[d] = d < c->g.nd ? reinterpret_cast<Real*>(b + q.off[d]) : nullptr;
  for (int k = 0; k < 3; k++) {
    a.u1[k] = reinterpret_cast<Real*>(b + q.u1[k]);
    a.u2[k] = s.d.kind == PIC_TWO_BODY ? reinterpret_cast<Real*>(b + q.u2[k]) : nullptr;
    a.dl[k] = s.d.kind == PIC_TWO_BODY ? reinterpret_cast<Real*>(b + q.dl[k]) : nullptr;
  }
  return a;
}

template <typename Real>
pic::FieldPtrs<Real> planes(void* base, int64_t plane) {
  pic::FieldPtrs<Real> f;
  Real* p = static_cast<Real*>(base);
  for (int a = 0; a < 3; a++) {
    f.E[a] = p + (0 + a) * plane;
    f.B[a] = p + (3 + a) * plane;
    f.J[a] = p + (6 + a) * plane;
  }
  return f;
}

int check_grad_ok(pic_ctx* c) {
  if (c->cfg.flags & (PIC_FLAG_FROZEN_FIELDS | PIC_FLAG_NO_DEPOSIT))
    return fail(c, PIC_EINVAL, "gradient runs need the coupled step (no frozen fields, deposit on)");
  if (c->sp.size() > 64) return fail(c, PIC_EINVAL, "gradient runs support at most 64 species");
  for (auto& s : c->sp)
    if (s->d.kind == PIC_MULTI_SHELL)
      return fail(c, PIC_EINVAL, "gradient runs do not take multi-shell species");
  return PIC_OK;
}

template <typename Real>
int grad_forward_t(pic_ctx* c, int64_t nsteps, int K) {
  if (!c->grad) c->grad = new GradState();
  GradState& G = *c->grad;
  G.ready = false;
  // one sort now (after a load), none during the run
  bool sorted = false;
  for (auto& s : c->sp)
    if (s->needs_sort) {
      if (pic::sort_by_tile(c->g, c->tile, c->ntiles, s->sort, s->n, c->stream, true))
        return fail(c, PIC_EHIP, "tile sort launch failed");
      s->needs_sort = false;
      s->listed_since_sort = 0.0;
      s->steps_since_sort = 0;
      sorted = true;
    }
  int rc = sorted ? update_occupancy(c) : PIC_OK;
  if (rc) return rc;
  rc = grad_buffers(c, nsteps, K);
  if (rc) return rc;
  G.nsteps = nsteps;
  G.K = K;
  G.step0 = c->step;
  G.rec0 = c->probe_rec;
  G.ck_step.assign(G.ck.size(), 0);
  const pic::LaserDev las = laser_dev(c);
  for (int64_t n = 0; n < nsteps; n++) {
    StepOpts o;
    SaveArg sa{nullptr, PIC_OK};
    const bool ck = n % K == 0;
    if (ck) {
      sa.buf = G.ck[n / K];
      G.ck_step[n / K] = c->step;
    }
    rc = advance_one<Real>(c, las, o, ck ? save_cb : nullptr, &sa);
    if (rc) return rc;
    if (sa.rc) return sa.rc;
  }
  if ((rc = snap_copy(c, G.final_state, true))) return rc;
  G.final_step = c->step;
  G.version = c->version;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, PIC_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
  G.ready = true;
  return PIC_OK;
}

template <typename Real>
int grad_backward_t(pic_ctx* c, const double* dprobe, pic_grad* out) {
  GradState& G = *c->grad;
  const GridInfo& g = c->g;
  const size_t rs = c->rsize;
  const int64_t nsteps = G.nsteps;
  // probe cotangent on the device (probe-major, nsteps per probe)
  const size_t nprobe = (size_t)c->nprobe;
  if (nprobe > 0) {
    const size_t bytes = nprobe * (size_t)nsteps * sizeof(double);
    if (bytes > G.dprobe_cap) {
      G.dprobe = static_cast<double*>(grad_alloc(c, bytes));
      if (!G.dprobe) return fail(c, PIC_ENOMEM, "device allocation failed");
      G.dprobe_cap = bytes;
    }
    HIPCHK(c, hipMemcpyAsync(G.dprobe, dprobe, bytes, hipMemcpyHostToDevice, c->stream));
  }
  // adjoint state starts at zero
  pic::FieldPtrs<Real> l = planes<Real>(G.lam_fields, g.plane);
  pic::launch_zero<Real>(l.E[0], 9 * g.plane, c->stream);
  for (int d = 0; d < g.nd; d++) {
    if (g.periodic[d]) continue;
    for (int t = 0; t < 2; t++) {
      pic::launch_zero<Real>(static_cast<Real*>(G.lam_mur_b[d][t]), face_bytes(c, d) / rs, c->stream);
      pic::launch_zero<Real>(static_cast<Real*>(G.lam_mur_e[d][t]), face_bytes(c, d) / rs, c->stream);
    }
  }
  for (size_t si = 0; si < c->sp.size(); si++) {
    pic::AdjState<Real> a = lam_state<Real>(c, si);
    for (int q = 0; q < 3; q++) {
      pic::launch_zero<Real>(a.off[q], a.n, c->stream);
      pic::launch_zero<Real>(a.dl[q], a.n, c->stream);
      pic::launch_zero<Real>(a.u1[q], a.n, c->stream);
      pic::launch_zero<Real>(a.u2[q], a.n, c->stream);
    }
  }
  pic::launch_zero<double>(G.dgrad, 256, c->stream);
  const pic::LaserDev las = laser_dev(c);
  Real* lEB[6] = {l.E[0], l.E[1], l.E[2], l.B[0], l.B[1], l.B[2]};
  Real* lJ[3] = {l.J[0], l.J[1], l.J[2]};
  const int64_t nseg = (nsteps + G.K - 1) / G.K;
  int rc;
  for (int64_t seg = nseg - 1; seg >= 0; seg--) {
    // re-run the segment, keeping the state at the start of each step
    if ((rc = snap_copy(c, G.ck[seg], false))) return rc;
    c->step = G.ck_step[seg];
    const int64_t n_lo = seg * G.K, n_hi = std::min<int64_t>(nsteps, n_lo + G.K);
    for (int64_t n = n_lo; n < n_hi; n++) {
      StepOpts o;
      o.record = false;
      SaveArg sa{G.slot[n - n_lo], PIC_OK};
      if ((rc = advance_one<Real>(c, las, o, save_cb, &sa))) return rc;
      if (sa.rc) return sa.rc;
    }
    for (int64_t n = n_hi - 1; n >= n_lo; n--) {
      void* slot = G.slot[n - n_lo];
      const int64_t step_n = G.ck_step[seg] + (n - n_lo);
      // probes recorded after step n
      pic::launch_probe_seed<Real>(l, c->nprobe, c->probe_comp, c->probe_idx, G.dprobe, nsteps,
                                   n, c->stream);
      // field update, in reverse
      pic::launch_b_half_adj<Real>(g, l, c->stream);
      for (int d = g.nd - 1; d >= 0; d--)
        if (!g.periodic[d])
          pic::launch_mur_high_e_adj<Real>(g, l, d, static_cast<Real*>(G.lam_mur_e[d][0]),
                                           static_cast<Real*>(G.lam_mur_e[d][1]), c->stream);
      pic::launch_fold_periodic<Real>(g, lEB, 3, c->stream, true);
      pic::launch_e_full_adj<Real>(g, l, c->stream);
      for (int d = g.nd - 1; d >= 0; d--)
        if (!g.periodic[d])
          pic::launch_save_high_e_adj<Real>(g, l, d, static_cast<Real*>(G.lam_mur_e[d][0]),
                                            static_cast<Real*>(G.lam_mur_e[d][1]), c->stream);
      for (int d = g.nd - 1; d >= 0; d--)
        if (!g.periodic[d])
          pic::launch_mur_low_b_adj<Real>(g, l, d, static_cast<Real*>(G.lam_mur_b[d][0]),
                                          static_cast<Real*>(G.lam_mur_b[d][1]), las, step_n,
                                          G.dgrad + 2 * c->sp.size(), c->stream);
      pic::launch_fold_periodic<Real>(g, lEB + 3, 3, c->stream, true);
      pic::launch_b_half_adj<Real>(g, l, c->stream);
      // J guard fold, transposed: guards take the adjoint of their alias
      pic::launch_fill_periodic<Real>(g, lJ, 3, c->stream, true);
      // particle cycles
      const Real* fslot = reinterpret_cast<const Real*>(static_cast<char*>(slot) + G.lay.fields);
      for (size_t si = 0; si < c->sp.size(); si++) {
        const SpeciesHost& s = *c->sp[si];
        if (s.n == 0) continue;
        const bool timed = record_event(c, PIC_TIMING_ADJOINT + (int)si, true);
        pic::AdjTiles tt{{c->tile[0], c->tile[1], c->tile[2]},
                         {c->ntiles[0], c->ntiles[1], c->ntiles[2]}};
        // one workgroup per tile when its LDS patch fits, else one thread
        // per particle with global atomics
        constexpr size_t kMaxAdjointLds = 160 * 1024;
        const bool tiled =
            c->tiled && pic::adjoint_lds_bytes(g, tt, sizeof(Real)) <= kMaxAdjointLds;
        const uint32_t* toff = tiled ? s.sort.tile_off : nullptr;
        pic::launch_adjoint_push<Real>(g, fslot, snap_state<Real>(c, slot, si),
                                       push_const<Real>(c, s), lam_state<Real>(c, si),
                                       static_cast<Real*>(G.lam_fields), G.dgrad + 2 * si,
                                       G.dgrad + kFarSlot, toff, tt, c->stream);
        if (timed) record_event(c, PIC_TIMING_ADJOINT + (int)si, false);
      }
      // E, B guard fill at the start of the step, transposed
      pic::launch_fold_periodic<Real>(g, lEB, 6, c->stream, true);
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, PIC_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
  // results
  std::vector<double> dg(256);
  HIPCHK(c, hipMemcpyAsync(dg.data(), G.dgrad, 256 * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (dg[kFarSlot] > 0.0)
    return fail(c, PIC_ERANGE,
                "the gradient run met two-body ions whose bodies are half a cell or more "
                "apart, which its reverse cycle does not cover");
  for (size_t si = 0; si < c->sp.size(); si++) {
    const pic_species_desc& d = c->sp[si]->d;
    const double dwc = dg[2 * si], dnu = dg[2 * si + 1];
    if (out->d_omega_c) out->d_omega_c[si] = dwc + d.nu_per_omega * dnu;
    if (out->d_nu) out->d_nu[si] = dnu;
  }
  if (out->d_env)
    for (int k = 0; k < c->cfg.laser.n_env; k++) out->d_env[k] = dg[2 * c->sp.size() + k];
  if (out->d_E || out->d_B) {
    std::vector<Real> plane(g.plane);
    const int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
    for (int comp = 0; comp < 6; comp++) {
      double* dst = comp < 3 ? (out->d_E ? out->d_E + comp * ncell : nullptr)
                             : (out->d_B ? out->d_B + (comp - 3) * ncell : nullptr);
      if (!dst) continue;
      HIPCHK(c, hipMemcpy(plane.data(), lEB[comp], g.plane * sizeof(Real), hipMemcpyDeviceToHost));
      for (int k = 0; k < g.n[2]; k++)
        for (int j = 0; j < g.n[1]; j++)
          for (int i = 0; i < g.n[0]; i++)
            dst[i + (int64_t)g.n[0] * (j + (int64_t)g.n[1] * k)] =
                (double)plane[g.origin + i + j * g.sy + k * g.sz];
    }
  }
  // back to the state at the end of the forward run
  if ((rc = snap_copy(c, G.final_state, false))) return rc;
  c->step = G.final_step;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PIC_OK;
}

template <typename Real>
int read_grad_particles_t(pic_ctx* c, size_t si, double* dx, double* ddelta, double* du1,
                          double* du2) {
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const SpeciesHost& s = *c->sp[si];
  const int64_t n = s.n;
  if (n == 0) return PIC_OK;
  pic::AdjState<Real> a = lam_state<Real>(c, si);
  std::vector<Real> buf(n);
  const int nd = c->g.nd;
  auto get = [&](Real* src, double* dst, int comp, int stride, double scale) -> int {
    HIPCHK(c, hipMemcpy(buf.data(), src, n * sizeof(Real), hipMemcpyDeviceToHost));
    for (int64_t p = 0; p < n; p++) dst[p * stride + comp] = scale * (double)buf[p];
    return PIC_OK;
  };
  int rc;
  const bool two = s.d.kind == PIC_TWO_BODY;
  // offsets are in cell units: d/dx = d/d(offset) / dx
  if (dx)
    for (int d = 0; d < nd; d++)
      if ((rc = get(a.off[d], dx, d, nd, 1.0 / c->cfg.dx[d]))) return rc;
  for (int q = 0; q < 3; q++) {
    if (du1 && (rc = get(a.u1[q], du1, q, 3, 1.0))) return rc;
    if (two && du2 && (rc = get(a.u2[q], du2, q, 3, 1.0))) return rc;
    if (two && ddelta && (rc = get(a.dl[q], ddelta, q, 3, 1.0))) return rc;
  }
  return PIC_OK;
}

}  // namespace

extern "C" {

int pic_grad_forward(pic_ctx* c, int32_t nsteps, int32_t checkpoint_every) {
  if (!c) return PIC_EINVAL;
  if (nsteps < 1 || checkpoint_every < 1)
    return fail(c, PIC_EINVAL, "nsteps and checkpoint_every must be >= 1");
  int rc = check_grad_ok(c);
  if (rc) return rc;
  if (c->nprobe > 0 && c->probe_rec + nsteps > c->cfg.max_probe_steps)
    return fail(c, PIC_EINVAL, "the probe record has no room for nsteps more steps");
  return c->prec == 32 ? grad_forward_t<float>(c, nsteps, checkpoint_every)
                       : grad_forward_t<double>(c, nsteps, checkpoint_every);
}

int pic_grad_backward(pic_ctx* c, const double* dprobe, pic_grad* out) {
  if (!c || !out) return PIC_EINVAL;
  if (!c->grad || !c->grad->ready)
    return fail(c, PIC_ESTATE, "pic_grad_backward needs a completed pic_grad_forward");
  if (c->nprobe > 0 && !dprobe) return fail(c, PIC_EINVAL, "dprobe is required with probes");
  for (size_t si = 0; si < c->sp.size(); si++)
    if (si >= c->grad->sp_n.size() || c->sp[si]->n != c->grad->sp_n[si])
      return fail(c, PIC_ESTATE, "species changed since pic_grad_forward");
  if (c->grad->final_step != c->step || c->grad->version != c->version)
    return fail(c, PIC_ESTATE, "the context was stepped or changed since pic_grad_forward");
  return c->prec == 32 ? grad_backward_t<float>(c, dprobe, out)
                       : grad_backward_t<double>(c, dprobe, out);
}

int pic_read_grad_particles(pic_ctx* c, int32_t sid, double* dx, double* ddelta, double* du1,
                            double* du2) {
  if (!c) return PIC_EINVAL;
  if (sid < 0 || sid >= (int32_t)c->sp.size()) return fail(c, PIC_ESTATE, "unknown species");
  if (!c->grad || !c->grad->ready || c->grad->lam_sp.size() != c->sp.size())
    return fail(c, PIC_ESTATE, "no gradient run");
  return c->prec == 32 ? read_grad_particles_t<float>(c, (size_t)sid, dx, ddelta, du1, du2)
                       : read_grad_particles_t<double>(c, (size_t)sid, dx, ddelta, du1, du2);
}

}  // extern "C"
