// tiled.h -- launch interface of the LDS-tiled particle kernel.
#pragma once

#include "pic_internal.h"

namespace pic {

constexpr int kTiledThreads = 512;
constexpr size_t kTiledMaxLds = 160 * 1024;  // LDS per CU on gfx950
constexpr int kQueueMax = 1024;              // queued general deposits per tile

// Tile geometry (per dimension; unresolved dimensions are 1).
struct TileGeom {
  int T[3];   // tile shape in cells
  int nt[3];  // tiles per dimension
  int nc[3];  // tiles of one colour per dimension (upper bound)
  int F[3];   // field patch extent: T + 4 (2-node apron each side)
  int Jd[3];  // current patch extent: T + 5 (2 below, 3 above)
  int qcap;   // LDS queue capacity for general (four-node) deposits
  int nd;     // resolved dimensions
};

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
// kernel for the particles they listed as outside their tile.  `list`
// holds room for every particle of the species; `nlist` is a scratch
// counter; `nlist_total` accumulates the listed count (diagnostics).
template <typename Real>
hipError_t launch_push_tiled(const GridInfo& g, const FieldPtrs<Real>& f, const SpeciesDev<Real>& s,
                             const PushConst<Real>& c, const TileGeom& t, const uint32_t* tile_off,
                             uint32_t* list, uint32_t* nlist, uint32_t* nlist_total,
                             uint32_t* err, hipStream_t st, DispatchHook hook = {});

}  // namespace pic
