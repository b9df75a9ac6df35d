// state.hip -- checkpoint and restart of a context: pic_save_state writes
// everything the next steps read into one self-describing host buffer,
// pic_load_state puts it back into a context created with the same grid,
// precision, flags and species.
//
// Layout of the buffer (all little-endian, as the host writes it):
//   Header
//   E, B, J: 9 guarded planes of the working precision (g.plane values each)
//   Mur history: for each non-periodic axis d, B then E, two planes each of
//     the face's values
//   per species: SpeciesRecord, then the tile offsets of its sorted order
//     (ntiles + 1 uint32, when its order is current), then the arrays cell
//     (uint32), offset[ndim], u1[3], and for two-body ions u2[3], delta[3],
//     then omega_c, weight (when carried) and load ids (PIC_FLAG_TRACK_IDS)
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ctx.h"

namespace {

constexpr char kMagic[8] = {'P', 'I', 'C', 'S', 'T', 'A', 'T', 'E'};
constexpr uint32_t kVersion = 1;

struct Header {
  char magic[8];
  uint32_t version, precision, ndim, nspecies;
  int64_t n[3];
  double dx[3];
  double dt;
  int64_t step, steps_since_sort;
  int64_t plane;
  uint32_t error_word, flags;
};

struct SpeciesRecord {
  int32_t kind, has_wc, has_w, needs_sort, has_ids, nshell;
  double q1, m1, q2, m2;
  int64_t n, steps_since_sort, ntiles;
  double max_w, listed_since_sort;
};

// What one piece of device memory contributes to the buffer.
struct Piece {
  void* dev;
  size_t bytes;
};

size_t face_values(const pic_ctx* c, int d) {
  const int a = d == 0 ? 1 : 0, b = d == 2 ? 1 : 2;
  return (size_t)c->g.n[a] * c->g.n[b];
}

// The device pieces of the state, in buffer order, with the species records.
void pieces_of(pic_ctx* c, std::vector<Piece>& fields, std::vector<SpeciesRecord>& recs,
               std::vector<std::vector<Piece>>& sp) {
  const size_t rs = c->rsize;
  fields.push_back({c->fields, 6 * (size_t)c->g.plane * rs});
  fields.push_back({c->jfield, 3 * (size_t)c->g.plane * rs});
  for (int d = 0; d < c->g.nd; d++) {
    if (c->g.periodic[d]) continue;
    const size_t fb = face_values(c, d) * rs;
    for (int t = 0; t < 2; t++) fields.push_back({c->mur_b[d][t], fb});
    for (int t = 0; t < 2; t++) fields.push_back({c->mur_e[d][t], fb});
  }
  for (auto& hp : c->sp) {
    SpeciesHost& s = *hp;
    const bool two = s.d.kind == PIC_TWO_BODY;
    SpeciesRecord r{};
    r.kind = s.d.kind;
    r.has_wc = s.has_wc;
    r.has_w = s.has_w;
    r.needs_sort = s.needs_sort;
    r.has_ids = s.ids != nullptr;
    r.nshell = s.nshell;
    r.q1 = s.d.q1;
    r.m1 = s.d.m1;
    r.q2 = s.d.q2;
    r.m2 = s.d.m2;
    r.n = s.n;
    r.steps_since_sort = s.steps_since_sort;
    r.ntiles = s.sort.ntiles;
    r.max_w = s.max_w;
    r.listed_since_sort = s.listed_since_sort;
    recs.push_back(r);
    std::vector<Piece> v;
    const size_t n = (size_t)s.n;
    if (!s.needs_sort) v.push_back({s.sort.tile_off, ((size_t)s.sort.ntiles + 1) * 4});
    v.push_back({s.cell, n * 4});
    for (int d = 0; d < c->g.nd; d++) v.push_back({s.off[d], n * rs});
    for (int a = 0; a < 3; a++) v.push_back({s.u1[a], n * rs});
    if (two) {
      for (int a = 0; a < 3; a++) v.push_back({s.u2[a], n * rs});
      for (int a = 0; a < 3; a++) v.push_back({s.dl[a], n * rs});
    }
    for (int k = 0; k < s.nshell; k++) {
      for (int a = 0; a < 3; a++) v.push_back({s.su2[k][a], n * rs});
      for (int a = 0; a < 3; a++) v.push_back({s.sdl[k][a], n * rs});
    }
    if (s.has_wc) v.push_back({s.wc, n * rs});
    if (s.has_w) v.push_back({s.w, n * rs});
    if (s.ids) v.push_back({s.ids, n * 8});
    sp.push_back(v);
  }
}

size_t total_bytes(const std::vector<Piece>& fields, const std::vector<std::vector<Piece>>& sp) {
  size_t b = sizeof(Header);
  for (const Piece& p : fields) b += p.bytes;
  for (const auto& v : sp) {
    b += sizeof(SpeciesRecord);
    for (const Piece& p : v) b += p.bytes;
  }
  return b;
}

}  // namespace

extern "C" {

int pic_save_state(pic_ctx* c, void* host_buf, size_t* bytes) {
  if (!c || !bytes) return c ? fail(c, PIC_EINVAL, "null argument") : PIC_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  harvest_pending_counts(c);  // the sort policy's counts of the last step
  std::vector<Piece> fields;
  std::vector<SpeciesRecord> recs;
  std::vector<std::vector<Piece>> sp;
  pieces_of(c, fields, recs, sp);
  const size_t need = total_bytes(fields, sp);
  if (!host_buf) {
    *bytes = need;
    return PIC_OK;
  }
  if (*bytes < need) {
    *bytes = need;
    return fail(c, PIC_EINVAL, "state buffer too small (size returned in *bytes)");
  }
  Header h{};
  std::memcpy(h.magic, kMagic, 8);
  h.version = kVersion;
  h.precision = (uint32_t)c->prec;
  h.ndim = (uint32_t)c->g.nd;
  h.nspecies = (uint32_t)c->sp.size();
  for (int d = 0; d < 3; d++) {
    h.n[d] = c->g.n[d];
    h.dx[d] = c->g.dx[d];
  }
  h.dt = c->cfg.dt;
  h.step = c->step;
  h.steps_since_sort = c->steps_since_sort;
  h.plane = c->g.plane;
  h.flags = c->cfg.flags;
  HIPCHK(c, hipMemcpy(&h.error_word, c->err, sizeof(uint32_t), hipMemcpyDeviceToHost));
  unsigned char* out = static_cast<unsigned char*>(host_buf);
  std::memcpy(out, &h, sizeof(h));
  size_t at = sizeof(h);
  for (const Piece& p : fields) {
    HIPCHK(c, hipMemcpy(out + at, p.dev, p.bytes, hipMemcpyDeviceToHost));
    at += p.bytes;
  }
  for (size_t si = 0; si < sp.size(); si++) {
    std::memcpy(out + at, &recs[si], sizeof(SpeciesRecord));
    at += sizeof(SpeciesRecord);
    for (const Piece& p : sp[si]) {
      if (p.bytes) HIPCHK(c, hipMemcpy(out + at, p.dev, p.bytes, hipMemcpyDeviceToHost));
      at += p.bytes;
    }
  }
  *bytes = need;
  return PIC_OK;
}

int pic_load_state(pic_ctx* c, const void* host_buf, size_t bytes) {
  if (!c || !host_buf) return c ? fail(c, PIC_EINVAL, "null argument") : PIC_EINVAL;
  c->version++;  // a gradient run started before this can no longer be reversed
  const unsigned char* in = static_cast<const unsigned char*>(host_buf);
  if (bytes < sizeof(Header)) return fail(c, PIC_EINVAL, "state buffer too short");
  Header h;
  std::memcpy(&h, in, sizeof(h));
  if (std::memcmp(h.magic, kMagic, 8) != 0 || h.version != kVersion)
    return fail(c, PIC_EINVAL, "not a libpic state buffer of this version");
  bool same = h.precision == (uint32_t)c->prec && h.ndim == (uint32_t)c->g.nd &&
              h.nspecies == (uint32_t)c->sp.size() && h.dt == c->cfg.dt &&
              h.plane == c->g.plane && h.flags == c->cfg.flags;
  for (int d = 0; d < 3; d++) same = same && h.n[d] == c->g.n[d] && h.dx[d] == c->g.dx[d];
  if (!same)
    return fail(c, PIC_EINVAL,
                "state of another grid, precision, flag set or species count than this context");
  // species records: kinds, charges and masses must match, counts must fit
  size_t at = sizeof(h) + 9 * (size_t)c->g.plane * c->rsize;
  for (int d = 0; d < c->g.nd; d++)
    if (!c->g.periodic[d]) at += 4 * face_values(c, d) * c->rsize;
  const size_t fields_end = at;
  std::vector<SpeciesRecord> recs(c->sp.size());
  for (size_t si = 0; si < c->sp.size(); si++) {
    if (at + sizeof(SpeciesRecord) > bytes) return fail(c, PIC_EINVAL, "state buffer too short");
    std::memcpy(&recs[si], in + at, sizeof(SpeciesRecord));
    const SpeciesRecord& r = recs[si];
    SpeciesHost& s = *c->sp[si];
    bool same = r.kind == s.d.kind && r.q1 == s.d.q1 && r.m1 == s.d.m1 && r.q2 == s.d.q2 &&
                r.m2 == s.d.m2 && r.nshell == s.nshell;
    if (!same)
      return fail(c, PIC_EINVAL, "species " + std::to_string(si) + " differs from the state's");
    if (r.n < 0 || r.n > s.cap)
      return fail(c, PIC_ENOMEM, "species " + std::to_string(si) + " capacity below the state's");
    if (r.ntiles != s.sort.ntiles || (r.has_ids != 0) != (s.ids != nullptr))
      return fail(c, PIC_EINVAL, "tiling or id tracking differs from the state's");
    const bool two = r.kind == PIC_TWO_BODY;
    size_t per = 4 + c->g.nd * c->rsize + 3 * c->rsize + (two ? 6 * c->rsize : 0) +
                 6 * (size_t)r.nshell * c->rsize +
                 (r.has_wc ? c->rsize : 0) + (r.has_w ? c->rsize : 0) + (r.has_ids ? 8 : 0);
    at += sizeof(SpeciesRecord) + (size_t)r.n * per +
          (r.needs_sort ? 0 : ((size_t)r.ntiles + 1) * 4);
  }
  if (at != bytes) return fail(c, PIC_EINVAL, "state buffer size does not match its contents");
  // per-particle omega_c / weight arrays, allocated as a load would
  for (size_t si = 0; si < c->sp.size(); si++) {
    SpeciesHost& s = *c->sp[si];
    if ((recs[si].has_wc && !s.has_wc) || (recs[si].has_w && !s.has_w)) {
      if (s.n > 0)
        return fail(c, PIC_ESTATE, "restore per-particle omega_c or weight into an empty species");
      int rc = prepare_optional(c, s, recs[si].has_wc, recs[si].has_w);
      if (rc) return rc;
    }
    if ((s.has_wc && !recs[si].has_wc) || (s.has_w && !recs[si].has_w))
      return fail(c, PIC_EINVAL, "the context carries per-particle arrays the state lacks");
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (size_t si = 0; si < c->sp.size(); si++) c->sp[si]->n = recs[si].n;  // sizes the pieces
  std::vector<Piece> fields;
  std::vector<SpeciesRecord> now;
  std::vector<std::vector<Piece>> sp;
  for (size_t si = 0; si < c->sp.size(); si++) c->sp[si]->needs_sort = recs[si].needs_sort != 0;
  pieces_of(c, fields, now, sp);
  at = sizeof(h);
  for (const Piece& p : fields) {
    HIPCHK(c, hipMemcpy(p.dev, in + at, p.bytes, hipMemcpyHostToDevice));
    at += p.bytes;
  }
  if (at != fields_end) return fail(c, PIC_EINVAL, "state layout mismatch");
  for (size_t si = 0; si < c->sp.size(); si++) {
    at += sizeof(SpeciesRecord);
    for (const Piece& p : sp[si]) {
      if (p.bytes) HIPCHK(c, hipMemcpy(p.dev, in + at, p.bytes, hipMemcpyHostToDevice));
      at += p.bytes;
    }
    SpeciesHost& s = *c->sp[si];
    const SpeciesRecord& r = recs[si];
    s.max_w = r.max_w;
    s.listed_since_sort = r.listed_since_sort;
    s.steps_since_sort = r.steps_since_sort;
  }
  HIPCHK(c, hipMemcpy(c->err, &h.error_word, sizeof(uint32_t), hipMemcpyHostToDevice));
  c->step = h.step;
  c->steps_since_sort = h.steps_since_sort;
  c->counts_pending = -1;
  c->residual_valid = false;
  return update_occupancy(c);  // the restored tile ranges
}

}  // extern "C"
