// tiled.h -- launch interface of the LDS-tiled particle kernel.
#pragma once

#include "pic_internal.h"

namespace pic {

constexpr int kTiledThreads = 512;
constexpr size_t kTiledMaxLds = 160 * 1024;  // LDS per CU on gfx950
constexpr int kQueueMax = 1024;              // queued general deposits per tile

// LDS row pitch (in values) for rows of `width` values such that a
// wavefront whose 64 lanes sit in `tx` consecutive cells of 64 / tx rows of
// one layer touches 64 distinct banks when they read the same relative
// node: the pitch is tx times an odd number (tx a divisor of 64 below 64;
// otherwise rows are packed).
constexpr int bank_pitch(int width, int tx) {
  if (tx <= 0 || tx >= 64 || 64 % tx != 0) return width;
  int m = (width + tx - 1) / tx;
  if (m % 2 == 0) m++;
  return tx * m;
}

// LDS layout of a tile's patches.  Field components are stored in pairs
// (Ex Ey | Ez Bx | By Bz) with the two rows of a pair side by side, which
// fills the row pitch that the bank rule asks for (24 values for an 8-cell
// tile row) with data instead of padding.  The three current components
// share each row, which is padded to the bank rule for 64-bit words (40
// words for an 8-cell tile: the 32 lanes of four 8-cell rows then cover the
// 64 banks once per relative node of the deposit's atomics).
struct PatchLayout {
  int F[3];    // field patch extent: T + 4 (2-node apron each side)
  int Jd[3];   // current patch extent: T + 5 (2 below, 3 above)
  int fpitch;  // field row pitch (2 components)
  int fplane;  // fpitch * F[1]
  int fpair;   // values of one component pair: fplane * F[2]
  int jpitch;  // current row pitch (3 components, packed)
  int jplane;  // jpitch * Jd[1]
  int nj;      // values of the current patch: jplane * Jd[2]
};

constexpr PatchLayout patch_layout(int tx, int ty, int tz, int nd) {
  PatchLayout L{};
  const int T[3] = {tx, ty, tz};
  for (int d = 0; d < 3; d++) {
    L.F[d] = d < nd ? T[d] + 4 : 1;
    L.Jd[d] = d < nd ? T[d] + 5 : 1;
  }
  L.fpitch = nd > 1 ? bank_pitch(2 * L.F[0], tx) : 2 * L.F[0];
  L.fplane = L.fpitch * L.F[1];
  L.fpair = L.fplane * L.F[2];
  L.jpitch = nd > 1 ? bank_pitch(3 * L.Jd[0], tx) : 3 * L.Jd[0];
  L.jplane = L.jpitch * L.Jd[1];
  L.nj = L.jplane * L.Jd[2];
  return L;
}

// Tile geometry (per dimension; unresolved dimensions are 1).
struct TileGeom {
  int T[3];       // tile shape in cells
  int nt[3];      // tiles per dimension
  int nc[3];      // tiles of one colour per dimension (upper bound)
  PatchLayout L;  // LDS layout of the patches
  int qcap;       // LDS queue capacity for general (four-node) deposits
  int nd;         // resolved dimensions
  // Sparse launches (most tiles empty): occ holds 8 per-colour counts, then
  // per colour the colour-local indices of the tiles that hold particles of
  // some species, in tile order (room for nc[0] nc[1] nc[2] each); the
  // dispatch of colour c runs occ_n[c] workgroups.  occ = nullptr: one
  // workgroup per tile of the colour.
  const uint32_t* occ = nullptr;
  uint32_t occ_n[8] = {};
};

// Fill the occupied-tile lists of a sparse launch (TileGeom::occ) from the
// sorted tile ranges of up to kOccSpecies species (one workgroup; the lists
// come out in tile order).
constexpr int kOccSpecies = 8;
hipError_t launch_occupied_tiles(const TileGeom& t, const uint32_t* const* tile_off, int nspecies,
                                 uint32_t* occ, hipStream_t st);

// Values per queued deposit: old and new position (resolved axes), charge,
// velocity along the unresolved axes.
constexpr int queue_vals(int nd) { return nd + 4; }

TileGeom make_tile_geom(const GridInfo& g, const int tile[3], const int ntiles[3], size_t rsize);
size_t tiled_lds_bytes(const TileGeom& t, size_t rsize);
bool tiled_supported(const GridInfo& g, const TileGeom& t, size_t rsize);

// Called on the host just before (start = true) and after (false) each
// colour dispatch is enqueued, e.g. to record timing events.
struct DispatchHook {
  void (*fn)(void* arg, bool start) = nullptr;
  void* arg = nullptr;
};

// Launch the 2^ndim colours of the tiled kernel for one species, then the
// kernel for the particles they listed as outside their tile (or, for
// two-body ions, with a body beyond [-1/2, 3/2) of its cell).  `list` holds
// room for every particle of the species; `defer` (two-body species; may
// be nullptr) likewise, for the ions each tile advances after its others;
// `nlist` is a scratch counter; `nlist_total` accumulates the listed count
// and `nfar` the ions listed for their separation (diagnostics and the
// sort policy).
template <typename Real>
hipError_t launch_push_tiled(const GridInfo& g, const FieldPtrs<Real>& f, const SpeciesDev<Real>& s,
                             const PushConst<Real>& c, const TileGeom& t, const uint32_t* tile_off,
                             uint32_t* list, uint32_t* defer, uint32_t* nlist,
                             uint32_t* nlist_total, uint32_t* nfar, uint32_t* err, hipStream_t st,
                             DispatchHook hook = {});

// A two-body species (i) and a point species (e) in one launch per tile
// colour: each workgroup advances both species' particles of its tile out
// of one LDS copy of the fields into one current patch (ci and ce must
// carry the same fixed-point scale), then the outside-tile kernel of each
// species.  defer_i as `defer` above for the ions; nlist holds two scratch
// counters; total_i, total_e accumulate the listed counts, nfar_i the ions
// listed for their separation.  `hook` brackets each shared colour
// dispatch.
template <typename Real>
hipError_t launch_push_tiled_pair(const GridInfo& g, const FieldPtrs<Real>& f,
                                  const SpeciesDev<Real>& si, const PushConst<Real>& ci,
                                  const uint32_t* tile_off_i, uint32_t* list_i,
                                  uint32_t* defer_i, const SpeciesDev<Real>& se,
                                  const PushConst<Real>& ce, const uint32_t* tile_off_e,
                                  uint32_t* list_e, const TileGeom& t, uint32_t* nlist,
                                  uint32_t* total_i, uint32_t* total_e, uint32_t* nfar_i,
                                  uint32_t* err, hipStream_t st, DispatchHook hook = {});

}  // namespace pic
