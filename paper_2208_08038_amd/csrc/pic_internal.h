// pic_internal.h -- device-side data layout and kernel launchers of libpic.
//
// HBM layout (one context):
//   fields   9 component planes (E, B, J), each (n_x + 2G)(n_y + 2G)(n_z + 2G)
//            values of the context precision, x fastest; G = 3 guard layers
//            on each side of every resolved dimension (unresolved: none).
//            Index of interior node (i, j, k): origin + i + j*sy + k*sz.
//   species  structure of arrays: packed cell (uint32: i | j << bx | k << (bx+by)),
//            offset[ndim], delta[3], u1[3], u2[3] (two-body), optional
//            omega_c and weight, all of the context precision; particles
//            grouped by tile.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pic.h"

namespace pic {

constexpr int kGuard = 3;

// Grid geometry shared by every kernel (passed by value).
struct GridInfo {
  int nd;
  int n[3];         // interior cells per dim (1 if unresolved)
  int g[3];         // guard layers per dim (kGuard if resolved, else 0)
  int st[3];        // storage extent per dim
  int64_t sy, sz;   // strides of y and z in the storage
  int64_t origin;   // storage index of interior node (0,0,0)
  int64_t plane;    // values per component plane
  int periodic[3];  // 1 if both faces periodic
  int pad;          // particle wall distance from non-periodic faces
  int bits[3];      // packed cell bits per dim
  double dx[3];
  double dt;
};

template <typename Real>
struct FieldPtrs {
  Real* E[3];
  Real* B[3];
  Real* J[3];
};

// One species' particle arrays (device pointers) and constants.
template <typename Real>
struct SpeciesDev {
  uint32_t* cell;
  Real* off[3];
  Real* dl[3];
  Real* u1[3];
  Real* u2[3];
  Real* wc;  // per-particle omega_c or nullptr
  Real* w;   // per-particle weight or nullptr
  int64_t n;
};

// Constants of the push of one species, precomputed on the host in FP64
// and rounded once to Real.
template <typename Real>
struct PushConst {
  Real dt, half_dt;
  Real idx[3];     // 1/dx
  Real a1, a2;     // (dt/2) q/m of body 1 and body 2
  Real m1, m2, inv_mc;
  Real f1, f2;     // m2/mc, m1/mc: body offsets from the centre of mass
  Real mr;         // reduced mass
  Real inv_q1, inv_q2;
  Real inv_ac2;    // 1/a_c^2 of the species, 0 for the harmonic bond
  // a_c derived from omega_c (Sec. 3.1, one Coulomb constant for every
  // ion): an ion with its own omega_c has 1/a_c^2 = ac_k * omega_c^{4/3};
  // 0 when a_c is fixed or the bond harmonic
  Real ac_k;
  Real omega_c, nu, nu_per_omega;
  Real qw1, qw2;   // q1 * weight, q2 * weight (species weight)
  Real weight;
  Real q1, q2;
  Real jf[3];      // -dx_d / (dt dV): Esirkepov prefactor per unit charge
  Real dxs[3];     // cell sizes (resolved dimensions)
  Real inv_dv;
  // power-of-two scale of the fixed-point LDS current patch: every deposit
  // term of this species times jscale is below 2^46 in magnitude
  Real jscale;
  int two_body;
  int deposit;
};

// Add the charge Q of one body at x (cell units, relative to the cell ci;
// any distance) to the FP64 density rho at integer nodes with the quadratic
// B-spline: the body is placed in the frame of the cell that holds it
// (wrapped along periodic axes; nodes b - 1 .. b + 2 must lie in the guarded
// storage, else nothing is added).  dv: cell volume.
template <int ND>
__device__ __forceinline__ void rho_add_body(const GridInfo& g, const int ci[3], const double xin[3],
                                             double Q, double dv, double* rho) {
  double x[3] = {0, 0, 0};
  int64_t base = g.origin;
  for (int d = 0; d < ND; d++) {
    const double k = floor(xin[d]);
    x[d] = xin[d] - k;
    int b = ci[d] + (int)k;
    if (g.periodic[d]) {
      b %= g.n[d];
      if (b < 0) b += g.n[d];
    }
    if (b < -2 || b > g.n[d]) return;
    base += (int64_t)b * (d == 0 ? 1 : (d == 1 ? g.sy : g.sz));
  }
  int i0[3] = {0, 0, 0};
  double w[3][3] = {{1, 0, 0}, {1, 0, 0}, {1, 0, 0}};
  for (int d = 0; d < ND; d++) {
    double f = floor(x[d] + 0.5), dd = x[d] - f;
    i0[d] = (int)f - 1;
    w[d][0] = 0.5 * (0.5 - dd) * (0.5 - dd);
    w[d][1] = 0.75 - dd * dd;
    w[d][2] = 0.5 * (0.5 + dd) * (0.5 + dd);
  }
  int nz = ND > 2 ? 3 : 1, ny = ND > 1 ? 3 : 1;
  for (int cz = 0; cz < nz; cz++)
    for (int cy = 0; cy < ny; cy++)
      for (int cx = 0; cx < 3; cx++) {
        double wt = w[0][cx] * w[1][cy] * w[2][cz];
        int64_t o = base + (i0[0] + cx) + (int64_t)(i0[1] + cy) * g.sy + (int64_t)(i0[2] + cz) * g.sz;
        if (wt != 0.0) unsafeAtomicAdd(rho + o, Q * wt / dv);
      }
}

// x^{4/3} for the softening length of an ion's own omega_c: FP32 through
// the hardware base-2 logarithm and exponential (about 1 ulp each), FP64 as
// x * cbrt(x).
__device__ __forceinline__ float pow43(float x) {
  return __builtin_amdgcn_exp2f(1.33333333f * __builtin_amdgcn_logf(x));
}
__device__ __forceinline__ double pow43(double x) { return x * cbrt(x); }

// 1/a_c^2 of an ion: its own when a_c derives from omega_c and the ion
// carries its own omega_c (Sec. 3.1 with one Coulomb constant: a_c^3
// proportional to 1/omega_c^2), else the species value.
template <typename Real>
__device__ __forceinline__ Real ion_inv_ac2(const PushConst<Real>& c, bool own_wc, Real wc) {
  return (own_wc && c.ac_k != Real(0)) ? c.ac_k * pow43(wc) : c.inv_ac2;
}

// Reflecting walls `pad` cells inside non-periodic faces act on each body
// of a two-body ion (Sec. 2: each body is a particle with its own position):
// a body past a wall is mirrored back into the box and its momentum
// component reversed; the centre of mass and delta follow the move D_i (in
// cells) of the mirrored body: R += (m_i / m_c) D_i, delta += +-D_i dx (+
// for the nucleus, - for the cloud).  offn: the centre's new offset
// relative to its old cell ci (before the crossing rule); dl, n1, n2: new
// delta and momenta.  Returns which bodies were mirrored: bit d for the
// nucleus along axis d, bit 4 + d for the cloud.
template <typename Real, int ND>
__device__ __forceinline__ unsigned two_body_walls(const GridInfo& g, const PushConst<Real>& c,
                                                   const int ci[3], Real offn[3], Real dl[3],
                                                   Real n1[3], Real n2[3]) {
  unsigned mask = 0u;
#pragma unroll
  for (int d = 0; d < ND; d++) {
    if (g.periodic[d]) continue;
    const Real lo = Real(g.pad - ci[d]), hi = Real(g.n[d] - g.pad - ci[d]);
    const Real sd = dl[d] * c.idx[d];
    const Real y1 = offn[d] + c.f1 * sd, y2 = offn[d] - c.f2 * sd;
    Real D1 = Real(0), D2 = Real(0);
    if (y1 < lo)
      D1 = Real(2) * (lo - y1);
    else if (y1 > hi)
      D1 = Real(2) * (hi - y1);
    if (y2 < lo)
      D2 = Real(2) * (lo - y2);
    else if (y2 > hi)
      D2 = Real(2) * (hi - y2);
    if (D1 != Real(0)) {
      mask |= 1u << d;
      n1[d] = -n1[d];
    }
    if (D2 != Real(0)) {
      mask |= 16u << d;
      n2[d] = -n2[d];
    }
    offn[d] += c.f2 * D1 + c.f1 * D2;
    dl[d] += (D1 - D2) * c.dxs[d];
  }
  return mask;
}

// Launchers (host).  All take the stream to launch on.
template <typename Real>
void launch_push(const GridInfo& g, const FieldPtrs<Real>& f, const SpeciesDev<Real>& s,
                 const PushConst<Real>& c, uint32_t* err, hipStream_t st);

template <typename Real>
void launch_push_list(const GridInfo& g, const FieldPtrs<Real>& f, const SpeciesDev<Real>& s,
                      const PushConst<Real>& c, const uint32_t* list, const uint32_t* count,
                      uint32_t* total, uint32_t* err, hipStream_t st);

template <typename Real>
void launch_zero(Real* p, int64_t n, hipStream_t st);

template <typename Real>
void launch_fill_periodic(const GridInfo& g, Real* const* comps, int ncomp, hipStream_t st,
                          bool reverse = false);

template <typename Real>
void launch_fold_periodic(const GridInfo& g, Real* const* comps, int ncomp, hipStream_t st,
                          bool reverse = false);

template <typename Real>
void launch_b_half(const GridInfo& g, const FieldPtrs<Real>& f, hipStream_t st);

template <typename Real>
void launch_e_full(const GridInfo& g, const FieldPtrs<Real>& f, hipStream_t st);

struct LaserDev {
  double a0, omega, t_env, waist, yc, zc, phase, t_delay;
  double cos_a, sin_a;  // direction of travel in the x-y plane
  int pol;
  int on;
  int oblique;
  int n_env;            // 0: sin^2 envelope; else cubic B-spline coefficients
  double h_env;         // knot spacing t_env / (n_env + 3)
  double env[64];
};

// One whole field step (B half, E full with J, B half, Mur faces and the
// x-min laser) in one pass, 1D and 2D: E and B read from fi and written to fo (distinct
// buffers; J from fi), the Mur history of the open low faces read from
// hist_in and written to hist_out (distinct).  fo's periodic guards are left
// stale (the next step refills them); its open-face guards get their Mur
// values.
template <typename Real>
hipError_t launch_yee_fused(const GridInfo& g, const FieldPtrs<Real>& fi, const FieldPtrs<Real>& fo,
                            Real* const hist_in[3][2], Real* const hist_out[3][2],
                            const LaserDev& las, int64_t step, hipStream_t st);

template <typename Real>
void launch_mur_low_b(const GridInfo& g, const FieldPtrs<Real>& f, int d, Real* prev0,
                      Real* prev1, const LaserDev& las, int64_t step, hipStream_t st);

template <typename Real>
void launch_save_high_e(const GridInfo& g, const FieldPtrs<Real>& f, int d, Real* save0,
                        Real* save1, hipStream_t st);

template <typename Real>
void launch_mur_high_e(const GridInfo& g, const FieldPtrs<Real>& f, int d, const Real* save0,
                       const Real* save1, hipStream_t st);

// diagnostics
// Adjoint (transposed) field operators of the gradient run; lE, lB, lJ in
// a FieldPtrs with the layout of the fields.
template <typename Real>
void launch_b_half_adj(const GridInfo& g, const FieldPtrs<Real>& l, hipStream_t st);
template <typename Real>
void launch_e_full_adj(const GridInfo& g, const FieldPtrs<Real>& l, hipStream_t st);
template <typename Real>
void launch_mur_low_b_adj(const GridInfo& g, const FieldPtrs<Real>& l, int d, Real* lprev0,
                          Real* lprev1, const LaserDev& las, int64_t step, double* genv,
                          hipStream_t st);
template <typename Real>
void launch_save_high_e_adj(const GridInfo& g, const FieldPtrs<Real>& l, int d, Real* ls0,
                            Real* ls1, hipStream_t st);
template <typename Real>
void launch_mur_high_e_adj(const GridInfo& g, const FieldPtrs<Real>& l, int d, Real* ls0,
                           Real* ls1, hipStream_t st);
template <typename Real>
void launch_probe_seed(const FieldPtrs<Real>& l, int nprobe, const int* comp,
                       const int64_t* index, const double* cot, int64_t nsteps, int64_t rec,
                       hipStream_t st);

template <typename Real>
void launch_rho(const GridInfo& g, const SpeciesDev<Real>& s, const PushConst<Real>& c,
                double* rho, hipStream_t st);

// Tile shape (cells) and tiles per dimension of a tile-sorted species.
struct TileGrid {
  int T[3];
  int nt[3];
};

// The charge density of launch_rho for a species sorted by tile (tile_off:
// the ntiles + 1 offsets of its sorted order); one workgroup per tile with
// an FP64 LDS patch of (T + 4) nodes per resolved dimension (tiles whose
// patch would exceed kRhoTiledMaxLds take launch_rho).
constexpr size_t kRhoTiledMaxLds = 64 * 1024;
size_t rho_tiled_lds(const GridInfo& g, const TileGrid& t);
template <typename Real>
void launch_rho_tiled(const GridInfo& g, const SpeciesDev<Real>& s, const PushConst<Real>& c,
                      const uint32_t* tile_off, const TileGrid& t, double* rho, hipStream_t st);

void launch_fold_periodic_f64(const GridInfo& g, double* rho, hipStream_t st);

// FP64 compensated reductions; each writes its results into out[] (device)
template <typename Real>
void launch_field_energy(const GridInfo& g, const FieldPtrs<Real>& f, double* partials,
                         int nblocks, double* out, hipStream_t st);

template <typename Real>
void launch_kinetic(const SpeciesDev<Real>& s, const PushConst<Real>& c, double* partials,
                    int nblocks, double* out /* 4: energy, px, py, pz */, hipStream_t st);

template <typename Real>
void launch_residual(const GridInfo& g, const FieldPtrs<Real>& f, const double* rho0,
                     const double* rho1, double* partials, int nblocks,
                     double* out /* 3: sum res^2, max |res|, sum drho^2 */, hipStream_t st);

template <typename Real>
void launch_probes(const GridInfo& g, const FieldPtrs<Real>& f, int nprobe, const int* comp,
                   const int64_t* index, Real* buf, int64_t max_steps, int64_t rec,
                   hipStream_t st);

int reduce_blocks();

}  // namespace pic
