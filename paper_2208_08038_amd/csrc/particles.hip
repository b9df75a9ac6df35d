// particles.hip -- the particle cycle: gather, internal force, relativistic
// Boris push, move and Esirkepov current deposit, for two-body macro-ions
// (An, Chen, Sheng, Zhang, arXiv 2208.08038, Sec. 2) and point particles.
//
// One lane advances one macro-particle through the whole cycle; the state
// is read once and written once (structure of arrays, coalesced).  Fields
// are read from the guarded Yee planes and the current is scattered with
// hardware floating-point atomics.
#include "pic_internal.h"

namespace pic {

namespace {

template <typename Real>
struct Weights {
  int i0;       // first node, relative to the particle's cell
  Real w[3];
};

// Quadratic B-spline weights on the integer-staggered nodes: nearest node
// i_n = floor(x + 1/2), d = x - i_n, weights at i_n-1, i_n, i_n+1.
template <typename Real>
__device__ __forceinline__ Weights<Real> weights_int(Real x) {
  Weights<Real> r;
  Real f = floor(x + Real(0.5));
  Real d = x - f;
  Real a = Real(0.5) - d, b = Real(0.5) + d;
  r.i0 = static_cast<int>(f) - 1;
  r.w[0] = Real(0.5) * a * a;
  r.w[1] = Real(0.75) - d * d;
  r.w[2] = Real(0.5) * b * b;
  return r;
}

// Same on the half-staggered nodes (positions i + 1/2, storage index i):
// nearest i_h = floor(x), d = x - i_h - 1/2.
template <typename Real>
__device__ __forceinline__ Weights<Real> weights_half(Real x) {
  Weights<Real> r;
  Real f = floor(x);
  Real d = x - f - Real(0.5);
  Real a = Real(0.5) - d, b = Real(0.5) + d;
  r.i0 = static_cast<int>(f) - 1;
  r.w[0] = Real(0.5) * a * a;
  r.w[1] = Real(0.75) - d * d;
  r.w[2] = Real(0.5) * b * b;
  return r;
}

template <typename Real, int ND>
__device__ __forceinline__ Real interp(const Real* __restrict__ F, int64_t base, int64_t sy,
                                       int64_t sz, const Weights<Real>& wx,
                                       const Weights<Real>& wy, const Weights<Real>& wz) {
  if constexpr (ND == 1) {
    const Real* p = F + base + wx.i0;
    return wx.w[0] * p[0] + wx.w[1] * p[1] + wx.w[2] * p[2];
  } else if constexpr (ND == 2) {
    Real s = 0;
#pragma unroll
    for (int b = 0; b < 3; b++) {
      const Real* p = F + base + wx.i0 + (int64_t)(wy.i0 + b) * sy;
      s += wy.w[b] * (wx.w[0] * p[0] + wx.w[1] * p[1] + wx.w[2] * p[2]);
    }
    return s;
  } else {
    Real s = 0;
#pragma unroll
    for (int c = 0; c < 3; c++) {
      Real t = 0;
#pragma unroll
      for (int b = 0; b < 3; b++) {
        const Real* p = F + base + wx.i0 + (int64_t)(wy.i0 + b) * sy + (int64_t)(wz.i0 + c) * sz;
        t += wy.w[b] * (wx.w[0] * p[0] + wx.w[1] * p[1] + wx.w[2] * p[2]);
      }
      s += wz.w[c] * t;
    }
    return s;
  }
}

// Gather E and B at a position x (cell units, relative to the cell whose
// storage index is `base`).  E_a is half-staggered along a; B_a along the
// two other axes.
template <typename Real, int ND>
__device__ __forceinline__ void gather(const FieldPtrs<Real>& f, int64_t base, int64_t sy,
                                       int64_t sz, const Real x[3], Real E[3], Real B[3]) {
  Weights<Real> n[3], h[3];
#pragma unroll
  for (int d = 0; d < 3; d++) {
    if (d < ND) {
      n[d] = weights_int(x[d]);
      h[d] = weights_half(x[d]);
    } else {
      n[d].i0 = 0;
      n[d].w[0] = 1;
      n[d].w[1] = 0;
      n[d].w[2] = 0;
      h[d] = n[d];
    }
  }
  E[0] = interp<Real, ND>(f.E[0], base, sy, sz, h[0], n[1], n[2]);
  E[1] = interp<Real, ND>(f.E[1], base, sy, sz, n[0], h[1], n[2]);
  E[2] = interp<Real, ND>(f.E[2], base, sy, sz, n[0], n[1], h[2]);
  B[0] = interp<Real, ND>(f.B[0], base, sy, sz, n[0], h[1], h[2]);
  B[1] = interp<Real, ND>(f.B[1], base, sy, sz, h[0], n[1], h[2]);
  B[2] = interp<Real, ND>(f.B[2], base, sy, sz, h[0], h[1], n[2]);
}

// Shape of a body at its old (x0) and new (x1) position on a common
// 4-node window starting at node `lo` (relative to the cell).  Returns
// false if the two nearest nodes are more than one node apart.
template <typename Real>
struct Window {
  int lo;
  Real S0[4], DS[4];
};

template <typename Real>
__device__ __forceinline__ bool window(Real x0, Real x1, Window<Real>& win) {
  Real f0 = floor(x0 + Real(0.5)), f1 = floor(x1 + Real(0.5));
  Real d0 = x0 - f0, d1 = x1 - f1;
  int i0 = static_cast<int>(f0), i1 = static_cast<int>(f1);
  int lo = min(i0, i1);
  int s0 = i0 - lo, s1 = i1 - lo;
  if (s0 > 1 || s1 > 1) return false;
  Real a0 = Real(0.5) - d0, b0 = Real(0.5) + d0;
  Real a1 = Real(0.5) - d1, b1 = Real(0.5) + d1;
  Real w0[3] = {Real(0.5) * a0 * a0, Real(0.75) - d0 * d0, Real(0.5) * b0 * b0};
  Real w1[3] = {Real(0.5) * a1 * a1, Real(0.75) - d1 * d1, Real(0.5) * b1 * b1};
  Real S0[4], S1[4];
  S0[0] = s0 ? Real(0) : w0[0];
  S0[1] = s0 ? w0[0] : w0[1];
  S0[2] = s0 ? w0[1] : w0[2];
  S0[3] = s0 ? w0[2] : Real(0);
  S1[0] = s1 ? Real(0) : w1[0];
  S1[1] = s1 ? w1[0] : w1[1];
  S1[2] = s1 ? w1[1] : w1[2];
  S1[3] = s1 ? w1[2] : Real(0);
  win.lo = lo - 1;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    win.S0[k] = S0[k];
    win.DS[k] = S1[k] - S0[k];
  }
  return true;
}

template <typename Real>
__device__ __forceinline__ void atomic_add(Real* p, Real v) {
  if (v != Real(0)) unsafeAtomicAdd(p, v);
}

// Esirkepov deposit of one body with charge Q (= q * weight) moving from
// x0 to x1 (cell units relative to the cell at storage index `base`).
// The current along a resolved axis is the running sum of the
// decomposition W_a = DS_a * (product of the other axes' shape averaged
// over the path); along an unresolved axis it is Q v times the
// path-averaged shape.
template <typename Real, int ND>
__device__ __forceinline__ bool deposit(const FieldPtrs<Real>& f, int64_t base, int64_t sy,
                                        int64_t sz, const Real x0[3], const Real x1[3], Real Q,
                                        const Real v[3], const PushConst<Real>& c) {
  Window<Real> w[ND];
#pragma unroll
  for (int d = 0; d < ND; d++)
    if (!window(x0[d], x1[d], w[d])) return false;
  const Real third = Real(1) / Real(3);
  if constexpr (ND == 1) {
    Real fx = Q * c.jf[0];
    Real fy = Q * v[1] * c.inv_dv, fz = Q * v[2] * c.inv_dv;
    Real C = 0;
    Real* Jx = f.J[0] + base + w[0].lo;
    Real* Jy = f.J[1] + base + w[0].lo;
    Real* Jz = f.J[2] + base + w[0].lo;
#pragma unroll
    for (int r = 0; r < 4; r++) {
      Real A = w[0].S0[r] + Real(0.5) * w[0].DS[r];
      if (r < 3) {
        C += w[0].DS[r];
        atomic_add(Jx + r, fx * C);
      }
      atomic_add(Jy + r, fy * A);
      atomic_add(Jz + r, fz * A);
    }
  } else if constexpr (ND == 2) {
    Real fx = Q * c.jf[0], fy = Q * c.jf[1], fz = Q * v[2] * c.inv_dv;
    Real Ax[4], Ay[4], By[4], Cx[3], Cy[3];
    Real cx = 0, cy = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) {
      Ax[k] = w[0].S0[k] + Real(0.5) * w[0].DS[k];
      Ay[k] = w[1].S0[k] + Real(0.5) * w[1].DS[k];
      By[k] = Real(0.5) * w[1].S0[k] + third * w[1].DS[k];
      if (k < 3) {
        cx += w[0].DS[k];
        cy += w[1].DS[k];
        Cx[k] = cx;
        Cy[k] = cy;
      }
    }
    int64_t b0 = base + w[0].lo + (int64_t)w[1].lo * sy;
#pragma unroll
    for (int s = 0; s < 4; s++) {
#pragma unroll
      for (int r = 0; r < 4; r++) {
        int64_t o = b0 + r + (int64_t)s * sy;
        if (r < 3) atomic_add(f.J[0] + o, fx * Cx[r] * Ay[s]);
        if (s < 3) atomic_add(f.J[1] + o, fy * Cy[s] * Ax[r]);
        atomic_add(f.J[2] + o, fz * (w[0].S0[r] * Ay[s] + w[0].DS[r] * By[s]));
      }
    }
  } else {
    Real fx = Q * c.jf[0], fy = Q * c.jf[1], fz = Q * c.jf[2];
    Real A[3][4], Bh[3][4], Cc[3][3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
      Real cs = 0;
#pragma unroll
      for (int k = 0; k < 4; k++) {
        A[d][k] = w[d].S0[k] + Real(0.5) * w[d].DS[k];
        Bh[d][k] = Real(0.5) * w[d].S0[k] + third * w[d].DS[k];
        if (k < 3) {
          cs += w[d].DS[k];
          Cc[d][k] = cs;
        }
      }
    }
    int64_t b0 = base + w[0].lo + (int64_t)w[1].lo * sy + (int64_t)w[2].lo * sz;
#pragma unroll
    for (int t = 0; t < 4; t++) {
#pragma unroll
      for (int s = 0; s < 4; s++) {
        // J_x: C_x(r) * [S0y (S0z + DSz/2) + DSy (S0z/2 + DSz/3)]
        Real Tx = w[1].S0[s] * A[2][t] + w[1].DS[s] * Bh[2][t];
#pragma unroll
        for (int r = 0; r < 4; r++) {
          int64_t o = b0 + r + (int64_t)s * sy + (int64_t)t * sz;
          if (r < 3) atomic_add(f.J[0] + o, fx * Cc[0][r] * Tx);
          if (s < 3) {
            Real Ty = w[0].S0[r] * A[2][t] + w[0].DS[r] * Bh[2][t];
            atomic_add(f.J[1] + o, fy * Cc[1][s] * Ty);
          }
          if (t < 3) {
            Real Tz = w[0].S0[r] * A[1][s] + w[0].DS[r] * Bh[1][s];
            atomic_add(f.J[2] + o, fz * Cc[2][t] * Tz);
          }
        }
      }
    }
  }
  return true;
}

template <typename Real>
__device__ __forceinline__ void boris_rotate_kick(Real um[3], Real a, const Real E[3],
                                                  const Real B[3], Real out[3]) {
  Real gm = sqrt(Real(1) + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
  Real k = a / gm;
  Real t[3] = {k * B[0], k * B[1], k * B[2]};
  Real t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
  Real sk = Real(2) / (Real(1) + t2);
  Real s[3] = {sk * t[0], sk * t[1], sk * t[2]};
  Real w[3] = {um[0] + (um[1] * t[2] - um[2] * t[1]), um[1] + (um[2] * t[0] - um[0] * t[2]),
               um[2] + (um[0] * t[1] - um[1] * t[0])};
  Real up[3] = {um[0] + (w[1] * s[2] - w[2] * s[1]), um[1] + (w[2] * s[0] - w[0] * s[2]),
                um[2] + (w[0] * s[1] - w[1] * s[0])};
#pragma unroll
  for (int q = 0; q < 3; q++) out[q] = up[q] + a * E[q];
}

// Reflecting walls `pad` cells inside non-periodic faces.  off: new offset
// relative to the old cell index ci (before the crossing rule).
template <typename Real>
__device__ __forceinline__ bool reflect(int periodic, int ci, int n, int pad, Real& off) {
  if (periodic) return false;
  int wl = pad, wr = n - pad;
  if (ci == wl && off < Real(0)) {
    off = -off;
    return true;
  }
  if (ci == wr - 1 && off > Real(1)) {
    off = Real(2) - off;
    return true;
  }
  if (ci == wr && off > Real(0)) {
    off = -off;
    return true;
  }
  return false;
}

// Integer cell-crossing rule; returns false if the new cell would leave
// the grid along a non-periodic axis.
template <typename Real>
__device__ __forceinline__ bool cross(int periodic, int n, int& ci, Real& off) {
  if (off >= Real(1)) {
    ci += 1;
    off -= Real(1);
  } else if (off < Real(0)) {
    ci -= 1;
    off += Real(1);
  }
  if (periodic) {
    if (ci >= n) ci -= n;
    if (ci < 0) ci += n;
    return true;
  }
  return ci >= 0 && ci < n;
}

template <typename Real>
__device__ __forceinline__ bool finite3(const Real v[3]) {
  return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]);
}

template <typename Real, int ND, bool TWO>
__global__ void __launch_bounds__(256) k_push(GridInfo g, FieldPtrs<Real> f, SpeciesDev<Real> s,
                                              PushConst<Real> c, uint32_t* err) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= s.n) return;
  const uint32_t packed = s.cell[p];
  int ci[3];
  ci[0] = packed & ((1u << g.bits[0]) - 1u);
  ci[1] = ND > 1 ? (packed >> g.bits[0]) & ((1u << g.bits[1]) - 1u) : 0;
  ci[2] = ND > 2 ? (packed >> (g.bits[0] + g.bits[1])) : 0;
  const int64_t base = g.origin + ci[0] + (int64_t)ci[1] * g.sy + (int64_t)ci[2] * g.sz;

  Real off[3] = {0, 0, 0};
#pragma unroll
  for (int d = 0; d < ND; d++) off[d] = s.off[d][p];
  Real u1[3], u2[3] = {0, 0, 0}, dl[3] = {0, 0, 0};
#pragma unroll
  for (int q = 0; q < 3; q++) u1[q] = s.u1[q][p];
  if constexpr (TWO) {
#pragma unroll
    for (int q = 0; q < 3; q++) {
      u2[q] = s.u2[q][p];
      dl[q] = s.dl[q][p];
    }
  }
  const Real W = s.w ? s.w[p] : Real(1);
  const Real qw1 = s.w ? c.q1 * W : c.qw1;

  // body positions (cell units, relative to the cell)
  Real x1[3] = {0, 0, 0}, x2[3] = {0, 0, 0};
  bool finite = finite3(u1) && finite3(u2) && finite3(dl);
  bool inside = true;
#pragma unroll
  for (int d = 0; d < ND; d++) {
    finite = finite && isfinite(off[d]);
    inside = inside && (off[d] >= Real(0)) && (off[d] <= Real(1));
    if constexpr (TWO) {
      Real sd = dl[d] * c.idx[d];
      inside = inside && (fabs(sd) < Real(0.5));
      x1[d] = off[d] + c.f1 * sd;
      x2[d] = off[d] - c.f2 * sd;
    } else {
      x1[d] = off[d];
    }
  }
  if (!finite || !inside) {
    // a particle that cannot be gathered safely is left untouched
    atomicOr(err, finite ? PIC_ERR_RANGE : PIC_ERR_NAN);
    return;
  }

  Real E1[3], B1[3];
  gather<Real, ND>(f, base, g.sy, g.sz, x1, E1, B1);
  Real n1[3], v1[3];
  if constexpr (TWO) {
    Real E2[3], B2[3];
    gather<Real, ND>(f, base, g.sy, g.sz, x2, E2, B2);
    const Real wc = s.wc ? s.wc[p] : c.omega_c;
    // softened Coulomb bond: F1 = -m_r w_c^2 delta (1 + |delta|^2/a_c^2)^{-3/2}
    Real r2 = dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2];
    Real soft = Real(1);
    if (c.inv_ac2 != Real(0)) {
      Real q = Real(1) + r2 * c.inv_ac2;
      Real rq = Real(1) / sqrt(q);
      soft = rq * rq * rq;
    }
    Real kf = -c.mr * wc * wc * soft;
#pragma unroll
    for (int q = 0; q < 3; q++) {
      Real F = kf * dl[q];
      E1[q] += F * c.inv_q1;
      E2[q] -= F * c.inv_q2;
    }
    Real um1[3], um2[3];
#pragma unroll
    for (int q = 0; q < 3; q++) {
      um1[q] = u1[q] + c.a1 * E1[q];
      um2[q] = u2[q] + c.a2 * E2[q];
    }
    const Real nu = c.nu + c.nu_per_omega * wc;
    if (nu > Real(0)) {
      // time-centred friction on the relative momentum; m1 u1 + m2 u2 kept
      Real D = (Real(1) - nu * c.half_dt) / (Real(1) + nu * c.half_dt);
#pragma unroll
      for (int q = 0; q < 3; q++) {
        Real V = (c.m1 * um1[q] + c.m2 * um2[q]) * c.inv_mc;
        Real w = (um1[q] - um2[q]) * D;
        um1[q] = V + c.f1 * w;
        um2[q] = V - c.f2 * w;
      }
    }
    Real n2[3];
    boris_rotate_kick(um1, c.a1, E1, B1, n1);
    boris_rotate_kick(um2, c.a2, E2, B2, n2);
    Real ig1 = Real(1) / sqrt(Real(1) + n1[0] * n1[0] + n1[1] * n1[1] + n1[2] * n1[2]);
    Real ig2 = Real(1) / sqrt(Real(1) + n2[0] * n2[0] + n2[1] * n2[1] + n2[2] * n2[2]);
    Real v2[3];
#pragma unroll
    for (int q = 0; q < 3; q++) {
      v1[q] = n1[q] * ig1;
      v2[q] = n2[q] * ig2;
    }
    // move: R += dt (m1 v1 + m2 v2)/m_c, delta += dt (v1 - v2)
    Real offn[3] = {0, 0, 0};
#pragma unroll
    for (int q = 0; q < 3; q++) dl[q] = dl[q] + c.dt * (v1[q] - v2[q]);
    bool range_ok = true;
#pragma unroll
    for (int d = 0; d < ND; d++) {
      offn[d] = off[d] + c.dt * (c.m1 * v1[d] + c.m2 * v2[d]) * c.inv_mc * c.idx[d];
      if (reflect(g.periodic[d], ci[d], g.n[d], g.pad, offn[d])) {
        n1[d] = -n1[d];
        n2[d] = -n2[d];
        dl[d] = -dl[d];
      }
    }
    Real y1[3] = {0, 0, 0}, y2[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < ND; d++) {
      Real sd = dl[d] * c.idx[d];
      range_ok = range_ok && (fabs(sd) < Real(0.5));
      y1[d] = offn[d] + c.f1 * sd;
      y2[d] = offn[d] - c.f2 * sd;
    }
    if (c.deposit) {
      const Real qw2 = s.w ? c.q2 * W : c.qw2;
      bool d1 = deposit<Real, ND>(f, base, g.sy, g.sz, x1, y1, qw1, v1, c);
      bool d2 = deposit<Real, ND>(f, base, g.sy, g.sz, x2, y2, qw2, v2, c);
      range_ok = range_ok && d1 && d2;
    }
    int cn[3] = {ci[0], ci[1], ci[2]};
#pragma unroll
    for (int d = 0; d < ND; d++) {
      int keep = cn[d];
      Real o = offn[d];
      if (cross(g.periodic[d], g.n[d], cn[d], o)) {
        offn[d] = o;
      } else {
        cn[d] = keep;
        range_ok = false;
      }
    }
    if (!range_ok) atomicOr(err, PIC_ERR_RANGE);
    if (!(finite3(n1) && finite3(n2) && finite3(dl))) atomicOr(err, PIC_ERR_NAN);
    uint32_t pk = (uint32_t)cn[0];
    if (ND > 1) pk |= (uint32_t)cn[1] << g.bits[0];
    if (ND > 2) pk |= (uint32_t)cn[2] << (g.bits[0] + g.bits[1]);
    s.cell[p] = pk;
#pragma unroll
    for (int d = 0; d < ND; d++) s.off[d][p] = offn[d];
#pragma unroll
    for (int q = 0; q < 3; q++) {
      s.u1[q][p] = n1[q];
      s.u2[q][p] = n2[q];
      s.dl[q][p] = dl[q];
    }
  } else {
    Real um[3];
#pragma unroll
    for (int q = 0; q < 3; q++) um[q] = u1[q] + c.a1 * E1[q];
    boris_rotate_kick(um, c.a1, E1, B1, n1);
    Real ig = Real(1) / sqrt(Real(1) + n1[0] * n1[0] + n1[1] * n1[1] + n1[2] * n1[2]);
#pragma unroll
    for (int q = 0; q < 3; q++) v1[q] = n1[q] * ig;
    Real y1[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < ND; d++) {
      y1[d] = off[d] + c.dt * v1[d] * c.idx[d];
      if (reflect(g.periodic[d], ci[d], g.n[d], g.pad, y1[d])) n1[d] = -n1[d];
    }
    bool range_ok = true;
    if (c.deposit) range_ok = deposit<Real, ND>(f, base, g.sy, g.sz, x1, y1, qw1, v1, c);
    int cn[3] = {ci[0], ci[1], ci[2]};
#pragma unroll
    for (int d = 0; d < ND; d++) {
      int keep = cn[d];
      Real o = y1[d];
      if (cross(g.periodic[d], g.n[d], cn[d], o)) {
        y1[d] = o;
      } else {
        cn[d] = keep;
        range_ok = false;
      }
    }
    if (!range_ok) atomicOr(err, PIC_ERR_RANGE);
    if (!finite3(n1)) atomicOr(err, PIC_ERR_NAN);
    uint32_t pk = (uint32_t)cn[0];
    if (ND > 1) pk |= (uint32_t)cn[1] << g.bits[0];
    if (ND > 2) pk |= (uint32_t)cn[2] << (g.bits[0] + g.bits[1]);
    s.cell[p] = pk;
#pragma unroll
    for (int d = 0; d < ND; d++) s.off[d][p] = y1[d];
#pragma unroll
    for (int q = 0; q < 3; q++) s.u1[q][p] = n1[q];
  }
}

}  // namespace

template <typename Real>
void launch_push(const GridInfo& g, const FieldPtrs<Real>& f, const SpeciesDev<Real>& s,
                 const PushConst<Real>& c, uint32_t* err, hipStream_t st) {
  if (s.n == 0) return;
  const int bs = 256;
  dim3 grid((unsigned)((s.n + bs - 1) / bs));
  if (c.two_body) {
    if (g.nd == 1) hipLaunchKernelGGL((k_push<Real, 1, true>), grid, bs, 0, st, g, f, s, c, err);
    if (g.nd == 2) hipLaunchKernelGGL((k_push<Real, 2, true>), grid, bs, 0, st, g, f, s, c, err);
    if (g.nd == 3) hipLaunchKernelGGL((k_push<Real, 3, true>), grid, bs, 0, st, g, f, s, c, err);
  } else {
    if (g.nd == 1) hipLaunchKernelGGL((k_push<Real, 1, false>), grid, bs, 0, st, g, f, s, c, err);
    if (g.nd == 2) hipLaunchKernelGGL((k_push<Real, 2, false>), grid, bs, 0, st, g, f, s, c, err);
    if (g.nd == 3) hipLaunchKernelGGL((k_push<Real, 3, false>), grid, bs, 0, st, g, f, s, c, err);
  }
}

template void launch_push<float>(const GridInfo&, const FieldPtrs<float>&,
                                 const SpeciesDev<float>&, const PushConst<float>&, uint32_t*,
                                 hipStream_t);
template void launch_push<double>(const GridInfo&, const FieldPtrs<double>&,
                                  const SpeciesDev<double>&, const PushConst<double>&, uint32_t*,
                                  hipStream_t);

}  // namespace pic
