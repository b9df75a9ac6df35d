// shells.h -- multi-shell ions: a nucleus and up to kMaxShell bound clouds,
// each cloud bound to the nucleus alone by the softened bond of Sec. 2 with
// its own charge, mass, restoring frequency and softening length (the
// extension the paper's summary names: the bound electrons of an ion in
// several components).  Stored as the centre of mass of all bodies (cell +
// offset), the nucleus momentum u0, and per cloud d_k = r_nucleus - r_k and
// its momentum u_k; one thread per ion.
#pragma once

#include "pic_internal.h"

namespace pic {

constexpr int kMaxShell = 4;

template <typename Real>
struct ShellDev {
  uint32_t* cell;
  Real* off[3];
  Real* u0[3];             // nucleus
  Real* dl[kMaxShell][3];  // d_k = r_nucleus - r_cloud_k (physical)
  Real* uk[kMaxShell][3];  // cloud k
  Real* w;                 // per-particle weight or nullptr
  int64_t n;
};

// Constants of a multi-shell species: body 0 is the nucleus, body k + 1
// cloud k.
template <typename Real>
struct ShellConst {
  Real q[kMaxShell + 1], inv_q[kMaxShell + 1], m[kMaxShell + 1];
  Real a[kMaxShell + 1];   // (dt/2) q / m
  Real fm[kMaxShell + 1];  // m / M (M: all bodies)
  Real qw[kMaxShell + 1];  // q * species weight
  Real kap[kMaxShell];     // bond stiffness m_r,k omega_k^2 (m_r,k of the nucleus-cloud pair)
  Real iac2[kMaxShell];    // 1 / a_k^2 (0: harmonic)
  Real pf0[kMaxShell], pfk[kMaxShell];  // m0 / (m0 + m_k), m_k / (m0 + m_k)
  Real inv_mp[kMaxShell];  // 1 / (m0 + m_k)
  Real inv_M;
  Real D;     // friction factor (1 - nu dt/2) / (1 + nu dt/2) on each pair
  int damp;   // nu > 0
  int K;      // number of clouds
};

template <typename Real>
hipError_t launch_push_shells(const GridInfo& g, const FieldPtrs<Real>& f, const ShellDev<Real>& s,
                              const ShellConst<Real>& sc, const PushConst<Real>& c,
                              uint32_t* err, hipStream_t st);

// The same step for a species sorted by tile (tile_off: the ntiles + 1
// offsets of its sorted order): one workgroup per tile, with an LDS
// current patch for the bodies whose frame cell lies in the tile; only for
// tiles whose patch (shells_tiled_lds) fits kShellsTiledMaxLds.
constexpr size_t kShellsTiledMaxLds = 64 * 1024;
size_t shells_tiled_lds(const GridInfo& g, const TileGrid& t);
template <typename Real>
hipError_t launch_push_shells_tiled(const GridInfo& g, const FieldPtrs<Real>& f,
                                    const ShellDev<Real>& s, const ShellConst<Real>& sc,
                                    const PushConst<Real>& c, const uint32_t* tile_off,
                                    const TileGrid& t, uint32_t* err, hipStream_t st);

// Device load of a multi-shell species (FP64 device arrays, layout as
// pic_load_particles: x n x ndim, delta and u2 n x 3K or nullptr, u1 n x 3,
// w n or nullptr), written at positions at .. at + n - 1 in load order.
// fm[b]: body b's mass over the ion's (b = 0 the nucleus); weight the
// species value for a missing w.  err as launch_load: [0] PIC_ERR_* bits,
// bytes 8..15 the bits of the largest |weight| loaded.
struct ShellLoad {
  const double* x;
  const double* delta;
  const double* u1;
  const double* u2;
  const double* w;
  int64_t n;
  double fm[kMaxShell + 1];
  double weight;
  int K;
};

template <typename Real>
void launch_load_shells(const GridInfo& g, const ShellLoad& src, const ShellDev<Real>& s,
                        int64_t at, int64_t* ids, uint32_t* err, hipStream_t st);

// charge density of every body (FP64 plane with guards, as launch_rho)
template <typename Real>
void launch_rho_shells(const GridInfo& g, const ShellDev<Real>& s, const ShellConst<Real>& sc,
                       const PushConst<Real>& c, double* rho, hipStream_t st);

}  // namespace pic
