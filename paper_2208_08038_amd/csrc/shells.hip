// shells.hip -- one step of a multi-shell ion (nucleus + K clouds, one bond
// each): the two-body step of Sec. 2 with a bond per cloud.  One thread per
// ion from HBM: every body is gathered at its own position in the frame of
// the cell that holds it, each bond adds +F_k / q0 to the nucleus' field
// and -F_k / q_k to cloud k's, the optional friction acts on each
// nucleus-cloud pair in turn (pair momentum kept), every body is
// Boris-pushed, the centre of mass moves with the mass-weighted velocities
// and d_k with v0 - v_k, the walls mirror each body, and each body deposits
// its own Esirkepov current.  A species sorted by tile is advanced one
// workgroup per tile: a body whose frame cell lies in the tile deposits into
// an FP64 LDS patch of the tile (its whole window lies there), added to the
// current planes with one global atomic per node; other bodies, and an
// unsorted species, deposit with global atomics.
#include <hip/hip_runtime.h>

#include "cycle.h"
#include "shells.h"

namespace pic {

namespace {

// Deposit of one body moving from x0 to x1 (cell units of the frame at
// `base`): the three-node window when it keeps its nearest node, else the
// general one.
template <typename Real, int ND, bool GLOBAL, typename JT>
__device__ __forceinline__ bool body_deposit(JT* const J[3], int base, int sy, int sz,
                                             const Real x0[3], const Real x1[3], Real Q,
                                             const Real v[3], const PushConst<Real>& c) {
  const Real* xs[2] = {x0, x1};
  int nn[3];
  if (common_node<Real, ND>(xs, 2, nn)) {
    Real d[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < ND; a++) d[a] = x1[a] - x0[a];
    deposit3<Real, ND, GLOBAL, JT, false>(J, base, sy, sz, nn, x0, d, Q, v, x0, d, Real(0), v,
                                          c);
    return true;
  }
  return deposit<Real, ND, GLOBAL, JT>(J, base, sy, sz, x0, x1, Q, v, c);
}

// Deposits of the global kernel: every body with global atomics.
template <typename Real, int ND>
struct GlobalDeposit {
  Real* J[3];
  int sy, sz;
  __device__ __forceinline__ bool operator()(int base, const Real x0[3], const Real x1[3], Real Q,
                                             const Real v[3], const int[3], const int[3],
                                             const PushConst<Real>& c) const {
    return body_deposit<Real, ND, true, Real>(J, base, sy, sz, x0, x1, Q, v, c);
  }
};

// Deposits of the tiled kernel: a body whose frame cell (the centre's cell
// ci shifted by k, unwrapped) lies in the tile's cells [lo, hi) adds into
// the LDS patch, whose nodes run from lo - 2 to hi + 2 (the deposit window
// of a body reaches two nodes below its cell and three above); any other
// body adds to the planes with global atomics.
template <typename Real, int ND>
struct TileDeposit {
  Real* J[3];
  int sy, sz;
  double* P[3];
  int psy, psz;
  int lo[3], hi[3];
  __device__ __forceinline__ bool operator()(int base, const Real x0[3], const Real x1[3], Real Q,
                                             const Real v[3], const int ci[3], const int k[3],
                                             const PushConst<Real>& c) const {
    bool in = true;
    int jb = 0;
#pragma unroll
    for (int d = 0; d < ND; d++) {
      const int cb = ci[d] + k[d];
      in = in && cb >= lo[d] && cb < hi[d];
      jb += (cb - lo[d] + 2) * (d == 0 ? 1 : (d == 1 ? psy : psz));
    }
    if (in) return body_deposit<Real, ND, false, double>(P, jb, psy, psz, x0, x1, Q, v, c);
    return body_deposit<Real, ND, true, Real>(J, base, sy, sz, x0, x1, Q, v, c);
  }
};

// The step of ion p; `dep` deposits each body's current.
template <typename Real, int ND, int K, typename Dep>
__device__ __forceinline__ void shell_ion(const GridInfo& g, const FieldPtrs<Real>& f,
                                          const ShellDev<Real>& s, const ShellConst<Real>& sc,
                                          const PushConst<Real>& c, uint32_t* err, int64_t p,
                                          const Dep& dep) {
  constexpr int NB = K + 1;
  int ci[3] = {0, 0, 0};
  decode_cell<ND>(g, s.cell[p], ci);
  Real off[3] = {0, 0, 0}, dl[K][3], u[NB][3];
  bool finite = true, inside = true;
#pragma unroll
  for (int d = 0; d < ND; d++) {
    off[d] = s.off[d][p];
    finite = finite && isfinite(off[d]);
    inside = inside && off[d] >= Real(0) && off[d] <= Real(1);
  }
#pragma unroll
  for (int q = 0; q < 3; q++) u[0][q] = s.u0[q][p];
#pragma unroll
  for (int k = 0; k < K; k++)
#pragma unroll
    for (int q = 0; q < 3; q++) {
      dl[k][q] = s.dl[k][q][p];
      u[k + 1][q] = s.uk[k][q][p];
    }
#pragma unroll
  for (int b = 0; b < NB; b++) finite = finite && finite3(u[b]);
#pragma unroll
  for (int k = 0; k < K; k++) finite = finite && finite3(dl[k]);
  if (!finite || !inside) {
    atomicOr(err, finite ? PIC_ERR_RANGE : PIC_ERR_NAN);  // left untouched
    return;
  }
  // body positions (cell units, relative to the centre's cell)
  Real x[NB][3];
#pragma unroll
  for (int b = 0; b < NB; b++)
#pragma unroll
    for (int d = 0; d < 3; d++) x[b][d] = Real(0);
#pragma unroll
  for (int d = 0; d < ND; d++) {
    Real r0 = off[d];
#pragma unroll
    for (int k = 0; k < K; k++) r0 += sc.fm[k + 1] * (dl[k][d] * c.idx[d]);
    x[0][d] = r0;
#pragma unroll
    for (int k = 0; k < K; k++) x[k + 1][d] = r0 - dl[k][d] * c.idx[d];
  }
#pragma unroll
  for (int b = 0; b < NB; b++)
    if (!body_in_range<Real, ND>(g, ci, x[b])) {
      atomicOr(err, PIC_ERR_RANGE);
      return;
    }
  const int sy = (int)g.sy, sz = (int)g.sz;
  int base[NB], kb[NB][3];
  Real bx[NB][3], E[NB][3], B[NB][3];
  // one body at a time (loop not unrolled: a single copy of the gather
  // keeps the live register set small); its results go to their body's
  // slots by selects
#pragma unroll 1
  for (int b = 0; b < NB; b++) {
    Real xb[3], ob[3], Eb[3], Bb[3];
    int kk[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
      xb[d] = x[0][d];
#pragma unroll
      for (int bb = 1; bb < NB; bb++) xb[d] = bb == b ? x[bb][d] : xb[d];
    }
    const int bs = body_frame<Real, ND>(g, ci, xb, ob, kk);
    gather<Real, ND>(f, bs, sy, sz, ob, Eb, Bb);
#pragma unroll
    for (int bb = 0; bb < NB; bb++) {
      base[bb] = bb == b ? bs : base[bb];
#pragma unroll
      for (int d = 0; d < 3; d++) {
        bx[bb][d] = bb == b ? ob[d] : bx[bb][d];
        kb[bb][d] = bb == b ? kk[d] : kb[bb][d];
        E[bb][d] = bb == b ? Eb[d] : E[bb][d];
        B[bb][d] = bb == b ? Bb[d] : B[bb][d];
      }
    }
  }
  // the bonds, as extra fields on the nucleus and on each cloud
#pragma unroll
  for (int k = 0; k < K; k++) {
    const Real r2 = dl[k][0] * dl[k][0] + dl[k][1] * dl[k][1] + dl[k][2] * dl[k][2];
    Real soft = Real(1);
    if (sc.iac2[k] != Real(0)) {
      const Real rq = rsqrt1(Real(1) + r2 * sc.iac2[k]);
      soft = rq * rq * rq;
    }
    const Real kf = -sc.kap[k] * soft;
#pragma unroll
    for (int q = 0; q < 3; q++) {
      const Real F = kf * dl[k][q];
      E[0][q] += F * sc.inv_q[0];
      E[k + 1][q] -= F * sc.inv_q[k + 1];
    }
  }
  Real um[NB][3];
#pragma unroll
  for (int b = 0; b < NB; b++)
#pragma unroll
    for (int q = 0; q < 3; q++) um[b][q] = u[b][q] + sc.a[b] * E[b][q];
  if (sc.damp) {
#pragma unroll
    for (int k = 0; k < K; k++)
#pragma unroll
      for (int q = 0; q < 3; q++) {
        const Real V = (sc.m[0] * um[0][q] + sc.m[k + 1] * um[k + 1][q]) * sc.inv_mp[k];
        const Real w = (um[0][q] - um[k + 1][q]) * sc.D;
        um[0][q] = V + sc.pfk[k] * w;
        um[k + 1][q] = V - sc.pf0[k] * w;
      }
  }
  Real nw[NB][3], v[NB][3];
#pragma unroll
  for (int b = 0; b < NB; b++) {
    boris_rotate_kick(um[b], sc.a[b], E[b], B[b], nw[b]);
    const Real ig = rsqrt1(Real(1) + nw[b][0] * nw[b][0] + nw[b][1] * nw[b][1] + nw[b][2] * nw[b][2]);
#pragma unroll
    for (int q = 0; q < 3; q++) v[b][q] = nw[b][q] * ig;
  }
  // move
#pragma unroll
  for (int k = 0; k < K; k++)
#pragma unroll
    for (int q = 0; q < 3; q++) dl[k][q] = dl[k][q] + c.dt * (v[0][q] - v[k + 1][q]);
  Real offn[3] = {0, 0, 0};
#pragma unroll
  for (int d = 0; d < ND; d++) {
    Real P = Real(0);
#pragma unroll
    for (int b = 0; b < NB; b++) P += sc.m[b] * v[b][d];
    offn[d] = off[d] + c.dt * P * sc.inv_M * c.idx[d];
  }
  // walls: a body past a wall is mirrored (moved by Dm cells) and its
  // momentum component reversed; the centre moves by (m_b / M) Dm; the
  // nucleus' move adds Dm dx to every d_k, cloud k's subtracts it from d_k
#pragma unroll
  for (int d = 0; d < ND; d++) {
    if (g.periodic[d]) continue;
    const Real lo = Real(g.pad - ci[d]), hi = Real(g.n[d] - g.pad - ci[d]);
    Real y[NB], Dm[NB];
    Real y0 = offn[d];
#pragma unroll
    for (int k = 0; k < K; k++) y0 += sc.fm[k + 1] * (dl[k][d] * c.idx[d]);
    y[0] = y0;
#pragma unroll
    for (int k = 0; k < K; k++) y[k + 1] = y0 - dl[k][d] * c.idx[d];
#pragma unroll
    for (int b = 0; b < NB; b++) {
      Dm[b] = Real(0);
      if (y[b] < lo)
        Dm[b] = Real(2) * (lo - y[b]);
      else if (y[b] > hi)
        Dm[b] = Real(2) * (hi - y[b]);
      if (Dm[b] != Real(0)) {
        nw[b][d] = -nw[b][d];
        offn[d] += sc.fm[b] * Dm[b];
      }
    }
#pragma unroll
    for (int k = 0; k < K; k++) dl[k][d] += (Dm[0] - Dm[k + 1]) * c.dxs[d];
  }
  // new body positions, relative to the centre's old cell
  Real yb[NB][3];
#pragma unroll
  for (int b = 0; b < NB; b++)
#pragma unroll
    for (int d = 0; d < 3; d++) yb[b][d] = Real(0);
#pragma unroll
  for (int d = 0; d < ND; d++) {
    Real r0 = offn[d];
#pragma unroll
    for (int k = 0; k < K; k++) r0 += sc.fm[k + 1] * (dl[k][d] * c.idx[d]);
    yb[0][d] = r0;
#pragma unroll
    for (int k = 0; k < K; k++) yb[k + 1][d] = r0 - dl[k][d] * c.idx[d];
  }
  bool range_ok = true;
#pragma unroll
  for (int b = 0; b < NB; b++) range_ok = range_ok && body_in_range<Real, ND>(g, ci, yb[b]);
  if (c.deposit) {
    const Real W = s.w ? s.w[p] : Real(0);
#pragma unroll 1
    for (int b = 0; b < NB; b++) {
      // body b's quantities, picked by selects (one copy of the deposit)
      Real ob[3], z[3] = {0, 0, 0}, vb[3];
      int kk[3], bs = base[0];
      Real Q = sc.qw[0], qb = sc.q[0];
#pragma unroll
      for (int d = 0; d < 3; d++) {
        ob[d] = bx[0][d];
        vb[d] = v[0][d];
        kk[d] = kb[0][d];
      }
      Real yy[3] = {yb[0][0], yb[0][1], yb[0][2]};
#pragma unroll
      for (int bb = 1; bb < NB; bb++) {
        const bool m = bb == b;
        bs = m ? base[bb] : bs;
        Q = m ? sc.qw[bb] : Q;
        qb = m ? sc.q[bb] : qb;
#pragma unroll
        for (int d = 0; d < 3; d++) {
          ob[d] = m ? bx[bb][d] : ob[d];
          vb[d] = m ? v[bb][d] : vb[d];
          kk[d] = m ? kb[bb][d] : kk[d];
          yy[d] = m ? yb[bb][d] : yy[d];
        }
      }
#pragma unroll
      for (int d = 0; d < ND; d++) z[d] = yy[d] - Real(kk[d]);
      if (s.w) Q = qb * W;
      range_ok = dep(bs, ob, z, Q, vb, ci, kk, c) && range_ok;
    }
  }
  int cn[3] = {ci[0], ci[1], ci[2]};
#pragma unroll
  for (int d = 0; d < ND; d++) {
    const int keep = cn[d];
    Real o = offn[d];
    if (cross(g.periodic[d], g.n[d], cn[d], o)) {
      offn[d] = o;
    } else {
      cn[d] = keep;
      range_ok = false;
    }
  }
  if (!range_ok) atomicOr(err, PIC_ERR_RANGE);
  bool fin = true;
#pragma unroll
  for (int b = 0; b < NB; b++) fin = fin && finite3(nw[b]);
#pragma unroll
  for (int k = 0; k < K; k++) fin = fin && finite3(dl[k]);
  if (!fin) atomicOr(err, PIC_ERR_NAN);
  s.cell[p] = encode_cell<ND>(g, cn);
#pragma unroll
  for (int d = 0; d < ND; d++) s.off[d][p] = offn[d];
#pragma unroll
  for (int q = 0; q < 3; q++) s.u0[q][p] = nw[0][q];
#pragma unroll
  for (int k = 0; k < K; k++)
#pragma unroll
    for (int q = 0; q < 3; q++) {
      s.dl[k][q][p] = dl[k][q];
      s.uk[k][q][p] = nw[k + 1][q];
    }
}

template <typename Real, int ND, int K>
__global__ void __launch_bounds__(256) k_push_shells(GridInfo g, FieldPtrs<Real> f,
                                                     ShellDev<Real> s, ShellConst<Real> sc,
                                                     PushConst<Real> c, uint32_t* err) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= s.n) return;
  const GlobalDeposit<Real, ND> dep{{f.J[0], f.J[1], f.J[2]}, (int)g.sy, (int)g.sz};
  shell_ion<Real, ND, K>(g, f, s, sc, c, err, p, dep);
}

// One workgroup per tile of the sorted order: its ions, with the LDS
// current patch of the tile (three FP64 component blocks of (T + 5) nodes
// per resolved dimension), then each non-zero patch node added to the
// planes with one global atomic.
template <typename Real, int ND, int K>
__global__ void __launch_bounds__(256) k_push_shells_tiled(GridInfo g, FieldPtrs<Real> f,
                                                           ShellDev<Real> s, ShellConst<Real> sc,
                                                           PushConst<Real> c,
                                                           const uint32_t* tile_off, TileGrid t,
                                                           uint32_t* err) {
  extern __shared__ double shell_patch[];
  const int64_t tile = blockIdx.x;
  const int64_t p0 = tile_off[tile], p1 = tile_off[tile + 1];
  if (p0 == p1) return;  // the whole block leaves before any barrier
  TileDeposit<Real, ND> dep;
  int P[3] = {1, 1, 1};
  int64_t r = tile;
#pragma unroll
  for (int d = 0; d < 3; d++) {
    dep.lo[d] = 0;
    dep.hi[d] = 1;
    if (d < ND) {
      const int tc = (int)(r % t.nt[d]);
      r /= t.nt[d];
      dep.lo[d] = tc * t.T[d];
      dep.hi[d] = min(dep.lo[d] + t.T[d], g.n[d]);
      P[d] = t.T[d] + 5;
    }
  }
  const int np = P[0] * P[1] * P[2];
  dep.psy = P[0];
  dep.psz = P[0] * P[1];
#pragma unroll
  for (int a = 0; a < 3; a++) {
    dep.J[a] = f.J[a];
    dep.P[a] = shell_patch + (int64_t)a * np;
  }
  dep.sy = (int)g.sy;
  dep.sz = (int)g.sz;
  for (int q = threadIdx.x; q < 3 * np; q += blockDim.x) shell_patch[q] = 0.0;
  __syncthreads();
  for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x)
    shell_ion<Real, ND, K>(g, f, s, sc, c, err, p, dep);
  __syncthreads();
  for (int q = threadIdx.x; q < np; q += blockDim.x) {
    // patch node q is grid node lo - 2 + its position (the planes' guards
    // reach 3 nodes out; nodes beyond are never written)
    int gi[3] = {0, 0, 0};
    int rem = q;
    bool ok = true;
#pragma unroll
    for (int d = 0; d < ND; d++) {
      gi[d] = dep.lo[d] - 2 + rem % P[d];
      rem /= P[d];
      ok = ok && gi[d] >= -kGuard && gi[d] < g.n[d] + kGuard;
    }
    if (!ok) continue;
    const int64_t gix = g.origin + gi[0] + (int64_t)gi[1] * g.sy + (int64_t)gi[2] * g.sz;
#pragma unroll
    for (int a = 0; a < 3; a++) {
      const double v = dep.P[a][q];
      if (v != 0.0) unsafeAtomicAdd(f.J[a] + gix, (Real)v);
    }
  }
}

// Device load, operation for operation as the host loader: position ->
// (packed cell, offset in the working precision), every body between the
// walls along walled axes, finite state.
template <typename Real, int ND, int K>
__global__ void __launch_bounds__(256) k_load_shells(GridInfo g, ShellLoad src, ShellDev<Real> s,
                                                     int64_t at, int64_t* ids, uint32_t* err) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= src.n) return;
  const int64_t q = at + p;
  uint32_t bad = 0;
  int ci[3] = {0, 0, 0};
  Real offr[3] = {0, 0, 0};
#pragma unroll
  for (int d = 0; d < ND; d++) {
    const double xv = src.x[p * ND + d];
    if (!isfinite(xv)) {
      bad |= PIC_ERR_NAN;
      continue;
    }
    const double xi = xv / g.dx[d];
    const double f = floor(xi);
    if (f < 0.0 || f >= (double)g.n[d]) {
      bad |= PIC_ERR_RANGE;
      continue;
    }
    int cc = (int)f;
    Real orr = (Real)(xi - f);
    if (orr >= Real(1)) {
      orr -= Real(1);
      cc += 1;
      if (cc >= g.n[d]) {
        if (g.periodic[d])
          cc -= g.n[d];
        else
          bad |= PIC_ERR_RANGE;
      }
    }
    ci[d] = cc;
    offr[d] = orr;
  }
  double dl[K][3];
#pragma unroll
  for (int k = 0; k < K; k++)
#pragma unroll
    for (int a = 0; a < 3; a++) {
      dl[k][a] = src.delta ? src.delta[3 * K * p + 3 * k + a] : 0.0;
      if (!isfinite(dl[k][a])) bad |= PIC_ERR_NAN;
    }
  // along walled axes every body lies between the walls
#pragma unroll
  for (int d = 0; d < ND; d++) {
    if (g.periodic[d] || bad) continue;
    double X0 = src.x[p * ND + d] / g.dx[d];
#pragma unroll
    for (int k = 0; k < K; k++) X0 += src.fm[k + 1] * dl[k][d] / g.dx[d];
    const double lo = g.pad, hi = g.n[d] - g.pad;
    bool ok = X0 >= lo && X0 <= hi;
#pragma unroll
    for (int k = 0; k < K; k++) {
      const double Xk = X0 - dl[k][d] / g.dx[d];
      ok = ok && Xk >= lo && Xk <= hi;
    }
    if (!ok) bad |= PIC_ERR_RANGE;
  }
  double u0[3], uk[K][3];
#pragma unroll
  for (int a = 0; a < 3; a++) {
    u0[a] = src.u1[3 * p + a];
    if (!isfinite(u0[a])) bad |= PIC_ERR_NAN;
  }
#pragma unroll
  for (int k = 0; k < K; k++)
#pragma unroll
    for (int a = 0; a < 3; a++) {
      uk[k][a] = src.u2 ? src.u2[3 * K * p + 3 * k + a] : u0[a];
      if (!isfinite(uk[k][a])) bad |= PIC_ERR_NAN;
    }
  if (bad) {
    atomicOr(err, bad);
    return;
  }
  uint32_t pk = (uint32_t)ci[0];
  if (ND > 1) pk |= (uint32_t)ci[1] << g.bits[0];
  if (ND > 2) pk |= (uint32_t)ci[2] << (g.bits[0] + g.bits[1]);
  s.cell[q] = pk;
#pragma unroll
  for (int d = 0; d < ND; d++) s.off[d][q] = offr[d];
#pragma unroll
  for (int a = 0; a < 3; a++) s.u0[a][q] = (Real)u0[a];
#pragma unroll
  for (int k = 0; k < K; k++)
#pragma unroll
    for (int a = 0; a < 3; a++) {
      s.dl[k][a][q] = (Real)dl[k][a];
      s.uk[k][a][q] = (Real)uk[k][a];
    }
  if (s.w) {
    const double w = src.w ? src.w[p] : src.weight;
    s.w[q] = (Real)w;
    atomicMax(reinterpret_cast<unsigned long long*>(err + 2),
              __builtin_bit_cast(unsigned long long, fabs(w)));
  }
  if (ids) ids[q] = q;
}

template <typename Real, int ND, int K>
__global__ void __launch_bounds__(256) k_rho_shells(GridInfo g, ShellDev<Real> s,
                                                    ShellConst<Real> sc, PushConst<Real> c,
                                                    double* rho) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= s.n) return;
  int ci[3] = {0, 0, 0};
  decode_cell<ND>(g, s.cell[p], ci);
  double dv = 1.0;
  for (int d = 0; d < ND; d++) dv *= g.dx[d];
  const double W = s.w ? (double)s.w[p] : 0.0;
  double x0[3] = {0, 0, 0};
  bool ok = true;
  for (int d = 0; d < ND; d++) {
    x0[d] = (double)s.off[d][p];
    for (int k = 0; k < K; k++) x0[d] += (double)sc.fm[k + 1] * ((double)s.dl[k][d][p] * (double)c.idx[d]);
    ok = ok && isfinite(x0[d]);
  }
  if (!ok) return;
  rho_add_body<ND>(g, ci, x0, s.w ? (double)sc.q[0] * W : (double)sc.qw[0], dv, rho);
  for (int k = 0; k < K; k++) {
    double x[3] = {0, 0, 0};
    for (int d = 0; d < ND; d++) x[d] = x0[d] - (double)s.dl[k][d][p] * (double)c.idx[d];
    rho_add_body<ND>(g, ci, x, s.w ? (double)sc.q[k + 1] * W : (double)sc.qw[k + 1], dv, rho);
  }
}

template <typename Real, int ND>
hipError_t push_nd(const GridInfo& g, const FieldPtrs<Real>& f, const ShellDev<Real>& s,
                   const ShellConst<Real>& sc, const PushConst<Real>& c, uint32_t* err,
                   hipStream_t st) {
  const unsigned nb = (unsigned)((s.n + 255) / 256);
  switch (sc.K) {
    case 1: hipLaunchKernelGGL((k_push_shells<Real, ND, 1>), nb, 256, 0, st, g, f, s, sc, c, err); break;
    case 2: hipLaunchKernelGGL((k_push_shells<Real, ND, 2>), nb, 256, 0, st, g, f, s, sc, c, err); break;
    case 3: hipLaunchKernelGGL((k_push_shells<Real, ND, 3>), nb, 256, 0, st, g, f, s, sc, c, err); break;
    case 4: hipLaunchKernelGGL((k_push_shells<Real, ND, 4>), nb, 256, 0, st, g, f, s, sc, c, err); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename Real, int ND>
hipError_t push_tiled_nd(const GridInfo& g, const FieldPtrs<Real>& f, const ShellDev<Real>& s,
                         const ShellConst<Real>& sc, const PushConst<Real>& c,
                         const uint32_t* tile_off, const TileGrid& t, uint32_t* err,
                         hipStream_t st) {
  int64_t ntiles = 1;
  for (int d = 0; d < ND; d++) ntiles *= t.nt[d];
  const size_t lds = shells_tiled_lds(g, t);
  if (lds > kShellsTiledMaxLds) return hipErrorInvalidValue;  // callers check first
  const dim3 nb((unsigned)ntiles);
  switch (sc.K) {
    case 1: hipLaunchKernelGGL((k_push_shells_tiled<Real, ND, 1>), nb, 256, lds, st, g, f, s, sc, c, tile_off, t, err); break;
    case 2: hipLaunchKernelGGL((k_push_shells_tiled<Real, ND, 2>), nb, 256, lds, st, g, f, s, sc, c, tile_off, t, err); break;
    case 3: hipLaunchKernelGGL((k_push_shells_tiled<Real, ND, 3>), nb, 256, lds, st, g, f, s, sc, c, tile_off, t, err); break;
    case 4: hipLaunchKernelGGL((k_push_shells_tiled<Real, ND, 4>), nb, 256, lds, st, g, f, s, sc, c, tile_off, t, err); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename Real, int ND>
void rho_nd(const GridInfo& g, const ShellDev<Real>& s, const ShellConst<Real>& sc,
            const PushConst<Real>& c, double* rho, hipStream_t st) {
  const unsigned nb = (unsigned)((s.n + 255) / 256);
  switch (sc.K) {
    case 1: hipLaunchKernelGGL((k_rho_shells<Real, ND, 1>), nb, 256, 0, st, g, s, sc, c, rho); break;
    case 2: hipLaunchKernelGGL((k_rho_shells<Real, ND, 2>), nb, 256, 0, st, g, s, sc, c, rho); break;
    case 3: hipLaunchKernelGGL((k_rho_shells<Real, ND, 3>), nb, 256, 0, st, g, s, sc, c, rho); break;
    case 4: hipLaunchKernelGGL((k_rho_shells<Real, ND, 4>), nb, 256, 0, st, g, s, sc, c, rho); break;
    default: break;
  }
}

}  // namespace

template <typename Real>
hipError_t launch_push_shells(const GridInfo& g, const FieldPtrs<Real>& f, const ShellDev<Real>& s,
                              const ShellConst<Real>& sc, const PushConst<Real>& c,
                              uint32_t* err, hipStream_t st) {
  if (s.n == 0) return hipSuccess;
  if (g.nd == 1) return push_nd<Real, 1>(g, f, s, sc, c, err, st);
  if (g.nd == 2) return push_nd<Real, 2>(g, f, s, sc, c, err, st);
  return push_nd<Real, 3>(g, f, s, sc, c, err, st);
}

size_t shells_tiled_lds(const GridInfo& g, const TileGrid& t) {
  size_t lds = 3 * sizeof(double);
  for (int d = 0; d < g.nd; d++) lds *= (size_t)(t.T[d] + 5);
  return lds;
}

template <typename Real>
hipError_t launch_push_shells_tiled(const GridInfo& g, const FieldPtrs<Real>& f,
                                    const ShellDev<Real>& s, const ShellConst<Real>& sc,
                                    const PushConst<Real>& c, const uint32_t* tile_off,
                                    const TileGrid& t, uint32_t* err, hipStream_t st) {
  if (s.n == 0) return hipSuccess;
  if (g.nd == 1) return push_tiled_nd<Real, 1>(g, f, s, sc, c, tile_off, t, err, st);
  if (g.nd == 2) return push_tiled_nd<Real, 2>(g, f, s, sc, c, tile_off, t, err, st);
  return push_tiled_nd<Real, 3>(g, f, s, sc, c, tile_off, t, err, st);
}

template <typename Real, int ND>
static void load_nd(const GridInfo& g, const ShellLoad& src, const ShellDev<Real>& s, int64_t at,
                    int64_t* ids, uint32_t* err, hipStream_t st) {
  const unsigned nb = (unsigned)((src.n + 255) / 256);
  switch (src.K) {
    case 1: hipLaunchKernelGGL((k_load_shells<Real, ND, 1>), nb, 256, 0, st, g, src, s, at, ids, err); break;
    case 2: hipLaunchKernelGGL((k_load_shells<Real, ND, 2>), nb, 256, 0, st, g, src, s, at, ids, err); break;
    case 3: hipLaunchKernelGGL((k_load_shells<Real, ND, 3>), nb, 256, 0, st, g, src, s, at, ids, err); break;
    case 4: hipLaunchKernelGGL((k_load_shells<Real, ND, 4>), nb, 256, 0, st, g, src, s, at, ids, err); break;
    default: break;
  }
}

template <typename Real>
void launch_load_shells(const GridInfo& g, const ShellLoad& src, const ShellDev<Real>& s,
                        int64_t at, int64_t* ids, uint32_t* err, hipStream_t st) {
  if (src.n <= 0) return;
  if (g.nd == 1) load_nd<Real, 1>(g, src, s, at, ids, err, st);
  if (g.nd == 2) load_nd<Real, 2>(g, src, s, at, ids, err, st);
  if (g.nd == 3) load_nd<Real, 3>(g, src, s, at, ids, err, st);
}

template <typename Real>
void launch_rho_shells(const GridInfo& g, const ShellDev<Real>& s, const ShellConst<Real>& sc,
                       const PushConst<Real>& c, double* rho, hipStream_t st) {
  if (s.n == 0) return;
  if (g.nd == 1) rho_nd<Real, 1>(g, s, sc, c, rho, st);
  if (g.nd == 2) rho_nd<Real, 2>(g, s, sc, c, rho, st);
  if (g.nd == 3) rho_nd<Real, 3>(g, s, sc, c, rho, st);
}

template hipError_t launch_push_shells<float>(const GridInfo&, const FieldPtrs<float>&,
                                              const ShellDev<float>&, const ShellConst<float>&,
                                              const PushConst<float>&, uint32_t*, hipStream_t);
template hipError_t launch_push_shells<double>(const GridInfo&, const FieldPtrs<double>&,
                                               const ShellDev<double>&, const ShellConst<double>&,
                                               const PushConst<double>&, uint32_t*, hipStream_t);
template hipError_t launch_push_shells_tiled<float>(const GridInfo&, const FieldPtrs<float>&,
                                                    const ShellDev<float>&,
                                                    const ShellConst<float>&,
                                                    const PushConst<float>&, const uint32_t*,
                                                    const TileGrid&, uint32_t*, hipStream_t);
template hipError_t launch_push_shells_tiled<double>(const GridInfo&, const FieldPtrs<double>&,
                                                     const ShellDev<double>&,
                                                     const ShellConst<double>&,
                                                     const PushConst<double>&, const uint32_t*,
                                                     const TileGrid&, uint32_t*, hipStream_t);
template void launch_load_shells<float>(const GridInfo&, const ShellLoad&,
                                        const ShellDev<float>&, int64_t, int64_t*, uint32_t*,
                                        hipStream_t);
template void launch_load_shells<double>(const GridInfo&, const ShellLoad&,
                                         const ShellDev<double>&, int64_t, int64_t*, uint32_t*,
                                         hipStream_t);
template void launch_rho_shells<float>(const GridInfo&, const ShellDev<float>&,
                                       const ShellConst<float>&, const PushConst<float>&, double*,
                                       hipStream_t);
template void launch_rho_shells<double>(const GridInfo&, const ShellDev<double>&,
                                        const ShellConst<double>&, const PushConst<double>&,
                                        double*, hipStream_t);

}  // namespace pic
