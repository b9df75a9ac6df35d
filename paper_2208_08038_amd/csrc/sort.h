// sort.h -- stable on-device ordering of particles by tile.
//
// Key = tile id of the particle's (centre-of-mass) cell.  The order is a
// stable LSD radix sort over digits of up to 9 bits of the key: within a
// tile the particles keep their previous relative order, so the
// permutation is unique and reproducible.  After a load the order within
// each tile is rebuilt as well: particles by their rank within their cell
// (first particle of every cell, then every cell's second, ...), cells
// ascending within each rank, so that the consecutive particles a
// wavefront advances sit in different cells (the deposit's LDS atomics of
// neighbouring lanes then hit different words) whatever order the caller
// loaded them in.  Every attribute array is then gathered through the
// permutation into an alternate buffer and the buffers are swapped.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>

#include "pic_internal.h"

namespace pic {

constexpr int kMaxAttr = 24;      // attributes moved by one gather launch
constexpr int kMaxSortAttr = 48;  // attributes of one species (gathered in launches of kMaxAttr)

struct SortBuffers {
  // key[0] (cap entries) is free between sorts: the tiled kernel keeps the
  // two-body ions it sets aside there (TileSpecies::defer)
  uint32_t* key[2] = {nullptr, nullptr};
  uint32_t* idx[2] = {nullptr, nullptr};
  uint32_t* hist = nullptr;     // 512 x blocks, digit-major
  uint32_t* scan_tmp = nullptr; // block sums of the scan levels
  uint32_t* tile_off = nullptr; // ntiles + 1 offsets of the sorted order
  int64_t ntiles = 0;
  int64_t cap = 0;
  int nattr = 0;
  void** attr[kMaxSortAttr] = {};   // pointers to the species' attribute pointers
  size_t elem[kMaxSortAttr] = {};   // element sizes
  void* alt[kMaxSortAttr] = {};     // alternate buffers
};

using AllocFn = std::function<void*(size_t)>;

// Allocate key/index/histogram buffers and tile offsets for `cap` particles.
int sort_alloc(const GridInfo& g, const int ntiles[3], int64_t cap, const AllocFn& alloc,
               SortBuffers& sb);

// Register one attribute array (pointer to the species' pointer) and
// allocate its alternate buffer.
int sort_add_attr(SortBuffers& sb, void** ptr, size_t elem, const AllocFn& alloc);

// Sort n particles by tile; swaps the registered attribute pointers.
// interleave: also order each tile by (rank within cell, cell), the rank
// counted in the present order and clamped at 255 (two more radix sorts
// and a rank pass; used after loads).  Falls back to the plain tile order
// when the (tile, cell) or (tile, rank) keys would not fit 32 bits.
int sort_by_tile(const GridInfo& g, const int tile[3], const int ntiles[3], SortBuffers& sb,
                 int64_t n, hipStream_t st, bool interleave = false);

}  // namespace pic
