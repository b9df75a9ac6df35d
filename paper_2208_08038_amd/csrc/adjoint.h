// adjoint.h -- launcher of the reverse-mode particle cycle (gradient run).
#pragma once

#include "pic_internal.h"

namespace pic {

// Particle arrays of one species as the adjoint kernel sees them: the
// stored state at the start of a step (cell, offsets, delta, u1, u2, and
// the species' per-particle omega_c and weight), or the adjoint of that
// state (offsets, delta, u1, u2 only).
template <typename Real>
using AdjState = SpeciesDev<Real>;

// Reverse the particle cycle of one step for one species (1D, 2D
// and 3D grids): reads the stored state `st`, the fields (E, B planes at the start
// of the step, guards filled, contiguous from `fields`, g.plane apart) and
// the adjoint current (planes 6..8 of `lam`, whose planes 0..5 are the
// adjoint E, B); updates the particle adjoint `lp` in place, adds the
// gather's transpose into the adjoint E, B, and adds d/d(omega_c) and
// d/d(friction rate) to dparam[0], dparam[1].  Two-body ions whose bodies
// are half a cell or more apart are not reversed; their number is added to
// *dfar.
// Tiles of the sorted particle order (cells per tile, tiles per dim).
struct AdjTiles {
  int T[3];
  int nt[3];
};

// Workgroups and LDS bytes of the tiled adjoint kernel (the launcher fails
// if the LDS does not fit a workgroup; the host checks first).
size_t adjoint_tiles(const GridInfo& g, const AdjTiles& tt);
size_t adjoint_lds_bytes(const GridInfo& g, const AdjTiles& tt, size_t rsize);

// With tile_off (the species' tile offsets of its last sort, which the
// gradient run keeps) one workgroup per tile accumulates the scatter in LDS;
// without, one thread per particle scatters with global atomics.
template <typename Real>
void launch_adjoint_push(const GridInfo& g, const Real* fields, const AdjState<Real>& st,
                         const PushConst<Real>& c, const AdjState<Real>& lp, Real* lam,
                         double* dparam, double* dfar, const uint32_t* tile_off,
                         const AdjTiles& tt, hipStream_t stream);

}  // namespace pic
