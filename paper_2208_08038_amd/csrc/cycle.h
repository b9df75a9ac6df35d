// cycle.h -- device code of one particle cycle, shared by the global and the
// LDS-tiled particle kernels: quadratic B-spline gather at the Yee
// staggers, softened bond force between nucleus and bound-electron cloud
// (An, Chen, Sheng, Zhang, arXiv 2208.08038, Sec. 2 and Sec. 3.1),
// optional friction on the relative momentum, relativistic Boris push of
// each body (Sec. 2), move of centre of mass and relative displacement,
// reflecting walls, integer cell crossing, Esirkepov current deposit.
//
// Indices into field planes and LDS patches are 32-bit (a plane holds
// fewer than 2^31 values; the host checks it), which keeps address
// arithmetic in single VGPRs.
#pragma once

#include <type_traits>

#include "pic_internal.h"

namespace pic {

template <typename Real>
struct Weights {
  int i0;  // first node, relative to the particle's cell
  Real w0, w1, w2;
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
  r.w0 = Real(0.5) * a * a;
  r.w1 = Real(0.75) - d * d;
  r.w2 = Real(0.5) * b * b;
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
  r.w0 = Real(0.5) * a * a;
  r.w1 = Real(0.75) - d * d;
  r.w2 = Real(0.5) * b * b;
  return r;
}

template <typename Real>
__device__ __forceinline__ Weights<Real> unit_weights() {
  Weights<Real> r;
  r.i0 = 0;
  r.w0 = Real(1);
  r.w1 = Real(0);
  r.w2 = Real(0);
  return r;
}

template <typename Real>
__device__ __forceinline__ Real row3(const Real* p, const Weights<Real>& wx) {
  return wx.w0 * p[0] + wx.w1 * p[1] + wx.w2 * p[2];
}

template <typename Real, int ND>
__device__ __forceinline__ Real interp(const Real* __restrict__ F, int base, int sy, int sz,
                                       const Weights<Real>& wx, const Weights<Real>& wy,
                                       const Weights<Real>& wz) {
  const Real* p = F + base + wx.i0;
  if constexpr (ND == 1) {
    return row3(p, wx);
  } else if constexpr (ND == 2) {
    p += wy.i0 * sy;
    return wy.w0 * row3(p, wx) + wy.w1 * row3(p + sy, wx) + wy.w2 * row3(p + 2 * sy, wx);
  } else {
    p += wy.i0 * sy + wz.i0 * sz;
    Real s = 0;
#pragma unroll
    for (int c = 0; c < 3; c++) {
      const Real* q = p + c * sz;
      Real t = wy.w0 * row3(q, wx) + wy.w1 * row3(q + sy, wx) + wy.w2 * row3(q + 2 * sy, wx);
      s += (c == 0 ? wz.w0 : (c == 1 ? wz.w1 : wz.w2)) * t;
    }
    return s;
  }
}

// Gather E and B at a position x (cell units, relative to the cell whose
// index is `base`).  E_a is half-staggered along a; B_a along the two
// other axes.
template <typename Real, int ND>
__device__ __forceinline__ void gather(const FieldPtrs<Real>& f, int base, int sy, int sz,
                                       const Real x[3], Real E[3], Real B[3]) {
  Weights<Real> n0 = weights_int(x[0]), h0 = weights_half(x[0]);
  Weights<Real> n1 = unit_weights<Real>(), h1 = unit_weights<Real>();
  Weights<Real> n2 = unit_weights<Real>(), h2 = unit_weights<Real>();
  if constexpr (ND > 1) {
    n1 = weights_int(x[1]);
    h1 = weights_half(x[1]);
  }
  if constexpr (ND > 2) {
    n2 = weights_int(x[2]);
    h2 = weights_half(x[2]);
  }
  E[0] = interp<Real, ND>(f.E[0], base, sy, sz, h0, n1, n2);
  E[1] = interp<Real, ND>(f.E[1], base, sy, sz, n0, h1, n2);
  E[2] = interp<Real, ND>(f.E[2], base, sy, sz, n0, n1, h2);
  B[0] = interp<Real, ND>(f.B[0], base, sy, sz, n0, h1, h2);
  B[1] = interp<Real, ND>(f.B[1], base, sy, sz, h0, n1, h2);
  B[2] = interp<Real, ND>(f.B[2], base, sy, sz, h0, h1, n2);
}

// Two positions whose stencils coincide (same first node for every
// stagger): one pass over the nodes accumulates both interpolants.
template <typename Real, int ND>
__device__ __forceinline__ void interp2(const Real* __restrict__ F, int base, int sy, int sz,
                                        const Weights<Real>& xa, const Weights<Real>& ya,
                                        const Weights<Real>& za, const Weights<Real>& xb,
                                        const Weights<Real>& yb, const Weights<Real>& zb,
                                        Real& ra, Real& rb) {
  const Real* p = F + base + xa.i0;
  if constexpr (ND > 1) p += ya.i0 * sy;
  if constexpr (ND > 2) p += za.i0 * sz;
  Real sa = 0, sb = 0;
  constexpr int NZ = ND > 2 ? 3 : 1, NY = ND > 1 ? 3 : 1;
#pragma unroll
  for (int cz = 0; cz < NZ; cz++) {
    Real ta = 0, tb = 0;
#pragma unroll
    for (int cy = 0; cy < NY; cy++) {
      const Real* q = p + cy * sy + cz * sz;
      Real v0 = q[0], v1 = q[1], v2 = q[2];
      Real wa = cy == 0 ? ya.w0 : (cy == 1 ? ya.w1 : ya.w2);
      Real wb = cy == 0 ? yb.w0 : (cy == 1 ? yb.w1 : yb.w2);
      ta += wa * (xa.w0 * v0 + xa.w1 * v1 + xa.w2 * v2);
      tb += wb * (xb.w0 * v0 + xb.w1 * v1 + xb.w2 * v2);
    }
    sa += (cz == 0 ? za.w0 : (cz == 1 ? za.w1 : za.w2)) * ta;
    sb += (cz == 0 ? zb.w0 : (cz == 1 ? zb.w1 : zb.w2)) * tb;
  }
  ra = sa;
  rb = sb;
}

// True when positions a and b have the same nearest integer and
// half-integer node along every resolved dimension.
template <typename Real, int ND>
__device__ __forceinline__ bool same_stencil(const Real xa[3], const Real xb[3]) {
  bool same = true;
#pragma unroll
  for (int d = 0; d < ND; d++)
    same = same && floor(xa[d] + Real(0.5)) == floor(xb[d] + Real(0.5)) &&
           floor(xa[d]) == floor(xb[d]);
  return same;
}

template <typename Real, int ND>
__device__ __forceinline__ void gather2(const FieldPtrs<Real>& f, int base, int sy, int sz,
                                        const Real xa[3], const Real xb[3], Real Ea[3],
                                        Real Ba[3], Real Eb[3], Real Bb[3]) {
  Weights<Real> na[3], ha[3], nb[3], hb[3];
#pragma unroll
  for (int d = 0; d < 3; d++) {
    if (d < ND) {
      na[d] = weights_int(xa[d]);
      ha[d] = weights_half(xa[d]);
      nb[d] = weights_int(xb[d]);
      hb[d] = weights_half(xb[d]);
    } else {
      na[d] = ha[d] = nb[d] = hb[d] = unit_weights<Real>();
    }
  }
  interp2<Real, ND>(f.E[0], base, sy, sz, ha[0], na[1], na[2], hb[0], nb[1], nb[2], Ea[0], Eb[0]);
  interp2<Real, ND>(f.E[1], base, sy, sz, na[0], ha[1], na[2], nb[0], hb[1], nb[2], Ea[1], Eb[1]);
  interp2<Real, ND>(f.E[2], base, sy, sz, na[0], na[1], ha[2], nb[0], nb[1], hb[2], Ea[2], Eb[2]);
  interp2<Real, ND>(f.B[0], base, sy, sz, na[0], ha[1], ha[2], nb[0], hb[1], hb[2], Ba[0], Bb[0]);
  interp2<Real, ND>(f.B[1], base, sy, sz, ha[0], na[1], ha[2], hb[0], nb[1], hb[2], Ba[1], Bb[1]);
  interp2<Real, ND>(f.B[2], base, sy, sz, ha[0], ha[1], na[2], hb[0], hb[1], nb[2], Ba[2], Bb[2]);
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
  Real w00 = Real(0.5) * a0 * a0, w01 = Real(0.75) - d0 * d0, w02 = Real(0.5) * b0 * b0;
  Real w10 = Real(0.5) * a1 * a1, w11 = Real(0.75) - d1 * d1, w12 = Real(0.5) * b1 * b1;
  Real S0[4], S1[4];
  S0[0] = s0 ? Real(0) : w00;
  S0[1] = s0 ? w00 : w01;
  S0[2] = s0 ? w01 : w02;
  S0[3] = s0 ? w02 : Real(0);
  S1[0] = s1 ? Real(0) : w10;
  S1[1] = s1 ? w10 : w11;
  S1[2] = s1 ? w11 : w12;
  S1[3] = s1 ? w12 : Real(0);
  win.lo = lo - 1;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    win.S0[k] = S0[k];
    win.DS[k] = S1[k] - S0[k];
  }
  return true;
}

// Add into a floating-point current (accumulator type JT, which may be
// wider than the arithmetic type): LDS patches take every term, global
// planes skip exact zeros (fewer atomics).
template <bool GLOBAL, typename JT, typename Real>
__device__ __forceinline__ void jadd(JT* p, Real v) {
  if constexpr (GLOBAL) {
    if (v != Real(0)) unsafeAtomicAdd(p, (JT)v);
  } else {
    unsafeAtomicAdd(p, (JT)v);
  }
}

// Add g_a X_a (+ g_b X_b with PAIR) into *p.  An integer JT is a 64-bit
// fixed-point LDS patch: the g carry the patch scale, a power of two the
// host chooses so that every term stays below 2^46 in magnitude.  Each
// product is formed exactly in FP64 inside an FMA whose running sum starts
// at 1.5 * 2^52: that sum has a unit ulp, so every FMA rounds its term to
// an integer (to nearest) and the low mantissa bits hold the integer sum
// of the rounded terms (valid below 2^51).  Integer adds are exact, so the
// patch sum does not depend on the order of the atomics, and 64-bit
// integer LDS atomics issue faster than FP64 ones on gfx950.
template <bool GLOBAL, bool PAIR, typename JT, typename Real>
__device__ __forceinline__ void jadd_terms(JT* p, Real ga, Real xa, Real gb, Real xb) {
  if constexpr (std::is_integral<JT>::value) {
    const double magic = 6755399441055744.0;
    double t = magic;
    if constexpr (PAIR) t = __builtin_fma((double)gb, (double)xb, t);
    t = __builtin_fma((double)ga, (double)xa, t);
    atomicAdd(reinterpret_cast<unsigned long long*>(p),
              static_cast<unsigned long long>(__builtin_bit_cast(long long, t) -
                                              __builtin_bit_cast(long long, magic)));
  } else {
    jadd<GLOBAL>(p, PAIR ? ga * xa + gb * xb : ga * xa);
  }
}

// Esirkepov deposit of one body with charge Q (= q * weight) moving from
// x0 to x1 (cell units relative to the cell at index `base`).  The current
// along a resolved axis is the running sum of the decomposition
// W_a = DS_a * (shape of the other axes averaged over the straight path);
// along an unresolved axis it is Q v times the path-averaged shape.
template <typename Real, int ND, bool GLOBAL, typename JT>
__device__ __forceinline__ bool deposit(JT* const J[3], int base, int sy, int sz,
                                        const Real x0[3], const Real x1[3], Real Q,
                                        const Real v[3], const PushConst<Real>& c) {
  const Real third = Real(1) / Real(3);
  // the charge carries the fixed-point scale into the prefactors
  if constexpr (std::is_integral<JT>::value) Q = Q * c.jscale;
  if constexpr (ND == 1) {
    Window<Real> wx;
    if (!window(x0[0], x1[0], wx)) return false;
    Real fx = Q * c.jf[0];
    Real fy = Q * v[1] * c.inv_dv, fz = Q * v[2] * c.inv_dv;
    Real C = 0;
    const int o = base + wx.lo;
#pragma unroll
    for (int r = 0; r < 4; r++) {
      Real A = wx.S0[r] + Real(0.5) * wx.DS[r];
      if (r < 3) {
        C += wx.DS[r];
        jadd_terms<GLOBAL, false>(J[0] + o + r, fx, C, Real(0), Real(0));
      }
      jadd_terms<GLOBAL, false>(J[1] + o + r, fy, A, Real(0), Real(0));
      jadd_terms<GLOBAL, false>(J[2] + o + r, fz, A, Real(0), Real(0));
    }
  } else if constexpr (ND == 2) {
    Window<Real> wx, wy;
    if (!window(x0[0], x1[0], wx) || !window(x0[1], x1[1], wy)) return false;
    Real fx = Q * c.jf[0], fy = Q * c.jf[1], fz = Q * v[2] * c.inv_dv;
    const int o = base + wx.lo + wy.lo * sy;
    // J_x = f_x C_x(r) (S0y + DSy/2)(s)
    {
      Real C = 0;
#pragma unroll
      for (int r = 0; r < 3; r++) {
        C += wx.DS[r];
        Real a = fx * C;
#pragma unroll
        for (int s = 0; s < 4; s++)
          jadd_terms<GLOBAL, false>(J[0] + o + r + s * sy, a,
                                    wy.S0[s] + Real(0.5) * wy.DS[s], Real(0), Real(0));
      }
    }
    // J_y = f_y C_y(s) (S0x + DSx/2)(r)
    {
      Real C = 0;
#pragma unroll
      for (int s = 0; s < 3; s++) {
        C += wy.DS[s];
        Real a = fy * C;
#pragma unroll
        for (int r = 0; r < 4; r++)
          jadd_terms<GLOBAL, false>(J[1] + o + r + s * sy, a,
                                    wx.S0[r] + Real(0.5) * wx.DS[r], Real(0), Real(0));
      }
    }
    // J_z = f_z [S0x (S0y + DSy/2) + DSx (S0y/2 + DSy/3)]
#pragma unroll
    for (int s = 0; s < 4; s++) {
      Real ay = wy.S0[s] + Real(0.5) * wy.DS[s];
      Real by = Real(0.5) * wy.S0[s] + third * wy.DS[s];
#pragma unroll
      for (int r = 0; r < 4; r++)
        jadd_terms<GLOBAL, false>(J[2] + o + r + s * sy, fz, wx.S0[r] * ay + wx.DS[r] * by,
                                  Real(0), Real(0));
    }
  } else {
    Window<Real> wx, wy, wz;
    if (!window(x0[0], x1[0], wx) || !window(x0[1], x1[1], wy) || !window(x0[2], x1[2], wz))
      return false;
    const int o = base + wx.lo + wy.lo * sy + wz.lo * sz;
    // J_x = f_x C_x(r) [S0y (S0z + DSz/2) + DSy (S0z/2 + DSz/3)](s, t)
    {
      const Real fx = Q * c.jf[0];
      const Real C0 = wx.DS[0], C1 = C0 + wx.DS[1], C2 = C1 + wx.DS[2];
      const Real g0 = fx * C0, g1 = fx * C1, g2 = fx * C2;
#pragma unroll
      for (int t = 0; t < 4; t++) {
        Real az = wz.S0[t] + Real(0.5) * wz.DS[t];
        Real bz = Real(0.5) * wz.S0[t] + third * wz.DS[t];
#pragma unroll
        for (int s = 0; s < 4; s++) {
          const Real X = wy.S0[s] * az + wy.DS[s] * bz;
          JT* p = J[0] + o + s * sy + t * sz;
          jadd_terms<GLOBAL, false>(p, g0, X, Real(0), Real(0));
          jadd_terms<GLOBAL, false>(p + 1, g1, X, Real(0), Real(0));
          jadd_terms<GLOBAL, false>(p + 2, g2, X, Real(0), Real(0));
        }
      }
    }
    // J_y = f_y C_y(s) [S0x (S0z + DSz/2) + DSx (S0z/2 + DSz/3)](r, t)
    {
      const Real fy = Q * c.jf[1];
      const Real C0 = wy.DS[0], C1 = C0 + wy.DS[1], C2 = C1 + wy.DS[2];
      const Real g0 = fy * C0, g1 = fy * C1, g2 = fy * C2;
#pragma unroll
      for (int t = 0; t < 4; t++) {
        Real az = wz.S0[t] + Real(0.5) * wz.DS[t];
        Real bz = Real(0.5) * wz.S0[t] + third * wz.DS[t];
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const Real X = wx.S0[r] * az + wx.DS[r] * bz;
          JT* p = J[1] + o + r + t * sz;
          jadd_terms<GLOBAL, false>(p, g0, X, Real(0), Real(0));
          jadd_terms<GLOBAL, false>(p + sy, g1, X, Real(0), Real(0));
          jadd_terms<GLOBAL, false>(p + 2 * sy, g2, X, Real(0), Real(0));
        }
      }
    }
    // J_z = f_z C_z(t) [S0x (S0y + DSy/2) + DSx (S0y/2 + DSy/3)](r, s)
    {
      const Real fz = Q * c.jf[2];
      const Real C0 = wz.DS[0], C1 = C0 + wz.DS[1], C2 = C1 + wz.DS[2];
      const Real g0 = fz * C0, g1 = fz * C1, g2 = fz * C2;
#pragma unroll
      for (int s = 0; s < 4; s++) {
        Real ay = wy.S0[s] + Real(0.5) * wy.DS[s];
        Real by = Real(0.5) * wy.S0[s] + third * wy.DS[s];
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const Real X = wx.S0[r] * ay + wx.DS[r] * by;
          JT* p = J[2] + o + r + s * sy;
          jadd_terms<GLOBAL, false>(p, g0, X, Real(0), Real(0));
          jadd_terms<GLOBAL, false>(p + sz, g1, X, Real(0), Real(0));
          jadd_terms<GLOBAL, false>(p + 2 * sz, g2, X, Real(0), Real(0));
        }
      }
    }
  }
  return true;
}

// Quadratic B-spline weights of a position x on the three nodes n-1, n, n+1.
template <typename Real>
__device__ __forceinline__ void shape3(Real x, int n, Real w[3]) {
  Real d = x - Real(n);
  Real a = Real(0.5) - d, b = Real(0.5) + d;
  w[0] = Real(0.5) * a * a;
  w[1] = Real(0.75) - d * d;
  w[2] = Real(0.5) * b * b;
}

// Old shape and shape change of a body on the 3-node window [n-1, n+1],
// from its old position x0 and its displacement dx.  The change of each
// quadratic B-spline weight factors through the displacement D (with
// d0 = x0 - n and s = d0 + d1 = 2 d0 + D):
//   S(n-1): -D (1 - s)/2,   S(n): -D s,   S(n+1): D (1 + s)/2,
// so a displacement much smaller than a cell keeps its relative precision
// (the difference of two nearly equal weights would lose it in FP32).
template <typename Real, int ND>
struct Win3 {
  Real S0[ND][3], DS[ND][3];
};

template <typename Real, int ND>
__device__ __forceinline__ void win3(const Real x0[3], const Real dx[3], const int nn[3],
                                     Win3<Real, ND>& w) {
#pragma unroll
  for (int d = 0; d < ND; d++) {
    shape3(x0[d], nn[d], w.S0[d]);
    const Real D = dx[d];
    const Real sum = Real(2) * (x0[d] - Real(nn[d])) + D;
    w.DS[d][0] = Real(-0.5) * D * (Real(1) - sum);
    w.DS[d][1] = -D * sum;
    w.DS[d][2] = Real(0.5) * D * (Real(1) + sum);
  }
}

// Esirkepov deposit when the nearest node does not change during the step
// (old and new positions of every body share the node n per dimension):
// the window is three nodes wide and the running sum along the motion has
// two non-zero terms (the third is the sum of the shape change, zero).
// Bodies are given by old position and displacement (see win3).  With
// PAIR the two bodies of an ion share the window and their terms are
// added in registers before one add per node.
// One current component of the 3D three-node deposit: along its axis AX the
// running sum of DS_AX has two non-zero terms C0 = DS(0), C1 = DS(0) + DS(1)
// (the third is the sum of the shape change, zero); across it the
// path-averaged shape S0_B (S0_E + DS_E/2) + DS_B (S0_E/2 + DS_E/3) over
// the transverse axes B < E.  The prefactor f and C are multiplied once
// (g = f C), not per node.  Strides: sb, se of the nodes along B and E,
// sa of the second node along AX.
template <typename Real, int ND, bool GLOBAL, typename JT, bool PAIR, int AX>
__device__ __forceinline__ void deposit3_axis(JT* Jc, int o, int sb, int se, int sa,
                                              const Win3<Real, ND>& a, const Win3<Real, ND>& b,
                                              Real fa, Real fb) {
  constexpr int B = AX == 0 ? 1 : 0, E = AX == 2 ? 1 : 2;
  const Real third = Real(1) / Real(3);
  const Real ga0 = fa * a.DS[AX][0], ga1 = fa * (a.DS[AX][0] + a.DS[AX][1]);
  Real gb0 = 0, gb1 = 0;
  if constexpr (PAIR) {
    gb0 = fb * b.DS[AX][0];
    gb1 = fb * (b.DS[AX][0] + b.DS[AX][1]);
  }
#pragma unroll
  for (int e = 0; e < 3; e++) {
    const Real Aa = a.S0[E][e] + Real(0.5) * a.DS[E][e];
    const Real Ba = Real(0.5) * a.S0[E][e] + third * a.DS[E][e];
    Real Ab = 0, Bb = 0;
    if constexpr (PAIR) {
      Ab = b.S0[E][e] + Real(0.5) * b.DS[E][e];
      Bb = Real(0.5) * b.S0[E][e] + third * b.DS[E][e];
    }
#pragma unroll
    for (int k = 0; k < 3; k++) {
      const Real Xa = a.S0[B][k] * Aa + a.DS[B][k] * Ba;
      Real Xb = 0;
      if constexpr (PAIR) Xb = b.S0[B][k] * Ab + b.DS[B][k] * Bb;
      JT* p = Jc + o + k * sb + e * se;
      jadd_terms<GLOBAL, PAIR>(p, ga0, Xa, gb0, Xb);
      jadd_terms<GLOBAL, PAIR>(p + sa, ga1, Xa, gb1, Xb);
    }
  }
}

template <typename Real, int ND, bool GLOBAL, typename JT, bool PAIR>
__device__ __forceinline__ void deposit3(JT* const J[3], int base, int sy, int sz,
                                         const int nn[3], const Real xa0[3], const Real da[3],
                                         Real Qa, const Real va[3], const Real xb0[3],
                                         const Real db[3], Real Qb, const Real vb[3],
                                         const PushConst<Real>& c) {
  const Real third = Real(1) / Real(3);
  // charges carry the fixed-point scale into the prefactors
  Real sc = Real(1);
  if constexpr (std::is_integral<JT>::value) sc = c.jscale;
  const Real qa = Qa * sc, qb = Qb * sc;
  Win3<Real, ND> a, b;
  win3<Real, ND>(xa0, da, nn, a);
  if constexpr (PAIR) win3<Real, ND>(xb0, db, nn, b);
  int o = base + nn[0] - 1;
  if constexpr (ND > 1) o += (nn[1] - 1) * sy;
  if constexpr (ND > 2) o += (nn[2] - 1) * sz;
  if constexpr (ND == 1) {
    Real fxa = qa * c.jf[0], fya = qa * va[1] * c.inv_dv, fza = qa * va[2] * c.inv_dv;
    Real fxb = 0, fyb = 0, fzb = 0;
    if constexpr (PAIR) {
      fxb = qb * c.jf[0];
      fyb = qb * vb[1] * c.inv_dv;
      fzb = qb * vb[2] * c.inv_dv;
    }
    Real Ca = 0, Cb = 0;
#pragma unroll
    for (int r = 0; r < 3; r++) {
      Real Aa = a.S0[0][r] + Real(0.5) * a.DS[0][r];
      Real Ab = 0;
      if constexpr (PAIR) Ab = b.S0[0][r] + Real(0.5) * b.DS[0][r];
      if (r < 2) {
        Ca += a.DS[0][r];
        if constexpr (PAIR) Cb += b.DS[0][r];
        jadd_terms<GLOBAL, PAIR>(J[0] + o + r, fxa, Ca, fxb, Cb);
      }
      jadd_terms<GLOBAL, PAIR>(J[1] + o + r, fya, Aa, fyb, Ab);
      jadd_terms<GLOBAL, PAIR>(J[2] + o + r, fza, Aa, fzb, Ab);
    }
  } else if constexpr (ND == 2) {
    Real fxa = qa * c.jf[0], fya = qa * c.jf[1], fza = qa * va[2] * c.inv_dv;
    Real fxb = 0, fyb = 0, fzb = 0;
    if constexpr (PAIR) {
      fxb = qb * c.jf[0];
      fyb = qb * c.jf[1];
      fzb = qb * vb[2] * c.inv_dv;
    }
    const Real gxa0 = fxa * a.DS[0][0], gxa1 = fxa * (a.DS[0][0] + a.DS[0][1]);
    const Real gya0 = fya * a.DS[1][0], gya1 = fya * (a.DS[1][0] + a.DS[1][1]);
    Real gxb0 = 0, gxb1 = 0, gyb0 = 0, gyb1 = 0;
    if constexpr (PAIR) {
      gxb0 = fxb * b.DS[0][0];
      gxb1 = fxb * (b.DS[0][0] + b.DS[0][1]);
      gyb0 = fyb * b.DS[1][0];
      gyb1 = fyb * (b.DS[1][0] + b.DS[1][1]);
    }
#pragma unroll
    for (int s2 = 0; s2 < 3; s2++) {
      Real Aya = a.S0[1][s2] + Real(0.5) * a.DS[1][s2];
      Real Bya = Real(0.5) * a.S0[1][s2] + third * a.DS[1][s2];
      Real Ayb = 0, Byb = 0;
      if constexpr (PAIR) {
        Ayb = b.S0[1][s2] + Real(0.5) * b.DS[1][s2];
        Byb = Real(0.5) * b.S0[1][s2] + third * b.DS[1][s2];
      }
      // J_x = f_x C_x(r) (S0y + DSy/2)(s)
      JT* px = J[0] + o + s2 * sy;
      jadd_terms<GLOBAL, PAIR>(px, gxa0, Aya, gxb0, Ayb);
      jadd_terms<GLOBAL, PAIR>(px + 1, gxa1, Aya, gxb1, Ayb);
#pragma unroll
      for (int r = 0; r < 3; r++) {
        Real Axa = a.S0[0][r] + Real(0.5) * a.DS[0][r];
        Real Axb = 0;
        if constexpr (PAIR) Axb = b.S0[0][r] + Real(0.5) * b.DS[0][r];
        // J_y = f_y C_y(s) (S0x + DSx/2)(r), for s < 2
        if (s2 < 2)
          jadd_terms<GLOBAL, PAIR>(J[1] + o + r + s2 * sy, s2 == 0 ? gya0 : gya1, Axa,
                                   s2 == 0 ? gyb0 : gyb1, Axb);
        // J_z = f_z [S0x (S0y + DSy/2) + DSx (S0y/2 + DSy/3)]
        Real Xa = a.S0[0][r] * Aya + a.DS[0][r] * Bya;
        Real Xb = 0;
        if constexpr (PAIR) Xb = b.S0[0][r] * Ayb + b.DS[0][r] * Byb;
        jadd_terms<GLOBAL, PAIR>(J[2] + o + r + s2 * sy, fza, Xa, fzb, Xb);
      }
    }
  } else {
    deposit3_axis<Real, ND, GLOBAL, JT, PAIR, 0>(J[0], o, sy, sz, 1, a, b, qa * c.jf[0],
                                                 qb * c.jf[0]);
    deposit3_axis<Real, ND, GLOBAL, JT, PAIR, 1>(J[1], o, 1, sz, sy, a, b, qa * c.jf[1],
                                                 qb * c.jf[1]);
    deposit3_axis<Real, ND, GLOBAL, JT, PAIR, 2>(J[2], o, 1, sy, sz, a, b, qa * c.jf[2],
                                                 qb * c.jf[2]);
  }
}

// Nearest node per dimension shared by all the given positions, if any.
template <typename Real, int ND>
__device__ __forceinline__ bool common_node(const Real* const* xs, int nx, int nn[3]) {
  bool same = true;
#pragma unroll
  for (int d = 0; d < 3; d++) nn[d] = 0;
#pragma unroll
  for (int d = 0; d < ND; d++) {
    Real f = floor(xs[0][d] + Real(0.5));
    for (int k = 1; k < nx; k++) same = same && floor(xs[k][d] + Real(0.5)) == f;
    nn[d] = static_cast<int>(f);
  }
  return same;
}

// Reciprocal and reciprocal square root of arguments >= 1 (Lorentz factors,
// softening and rotation denominators).  FP32 uses the hardware
// approximations (within 1 ulp) instead of the correctly rounded
// division and square-root sequences; FP64 keeps the correctly rounded ones.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
__device__ __forceinline__ float rsqrt1(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt1(double x) { return 1.0 / sqrt(x); }

template <typename Real>
__device__ __forceinline__ void boris_rotate_kick(const Real um[3], Real a, const Real E[3],
                                                  const Real B[3], Real out[3]) {
  Real k = a * rsqrt1(Real(1) + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
  Real t0 = k * B[0], t1 = k * B[1], t2 = k * B[2];
  Real tt = t0 * t0 + t1 * t1 + t2 * t2;
  Real sk = Real(2) * recip(Real(1) + tt);
  Real s0 = sk * t0, s1 = sk * t1, s2 = sk * t2;
  Real w0 = um[0] + (um[1] * t2 - um[2] * t1);
  Real w1 = um[1] + (um[2] * t0 - um[0] * t2);
  Real w2 = um[2] + (um[0] * t1 - um[1] * t0);
  out[0] = um[0] + (w1 * s2 - w2 * s1) + a * E[0];
  out[1] = um[1] + (w2 * s0 - w0 * s2) + a * E[1];
  out[2] = um[2] + (w0 * s1 - w1 * s0) + a * E[2];
}

// Internal force, friction and Boris push of both bodies of an ion
// (Sec. 2).  E1, B1 and E2, B2 are the fields gathered at the bodies; the
// softened Coulomb force F1 = -m_r w_c^2 delta (1 + |delta|^2/a_c^2)^{-3/2}
// acts as extra E (+F/q1 on the nucleus, -F/q2 on the cloud); the friction
// (rate nu + nu_per_omega w_c) is time-centred on the relative momentum
// between the half kicks and keeps m1 u1 + m2 u2.  n1, n2: new momenta.
// A body at x (cell units, relative to its ion's cell) in [-1/2, 3/2)
// along an axis keeps its gather stencils within two nodes of the cell and
// its deposit window (over a step of less than a cell) within two nodes
// below and three above: the reach of a tile's field and current patches and
// of the guard layers.  An ion with both bodies so placed is advanced in the
// ion's cell frame (the tiled kernel or the HBM pass); bodies farther apart
// take the far-body path, each in its own cell frame.
template <typename Real>
__device__ __forceinline__ bool body_near(Real x) {
  return x >= Real(-0.5) && x < Real(1.5);
}

template <typename Real>
__device__ __forceinline__ void two_body_kick(const PushConst<Real>& c, Real wc, Real iac2,
                                              const Real dl[3], const Real u1[3],
                                              const Real u2[3], Real E1[3], const Real B1[3],
                                              Real E2[3], const Real B2[3], Real n1[3],
                                              Real n2[3]) {
  const Real r2 = dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2];
  Real soft = Real(1);
  if (iac2 != Real(0)) {
    const Real rq = rsqrt1(Real(1) + r2 * iac2);
    soft = rq * rq * rq;
  }
  const Real kf = -c.mr * wc * wc * soft;
  Real um1[3], um2[3];
#pragma unroll
  for (int q = 0; q < 3; q++) {
    const Real F = kf * dl[q];
    E1[q] += F * c.inv_q1;
    E2[q] -= F * c.inv_q2;
    um1[q] = u1[q] + c.a1 * E1[q];
    um2[q] = u2[q] + c.a2 * E2[q];
  }
  const Real nu = c.nu + c.nu_per_omega * wc;
  if (nu > Real(0)) {
    const Real D = (Real(1) - nu * c.half_dt) * recip(Real(1) + nu * c.half_dt);
#pragma unroll
    for (int q = 0; q < 3; q++) {
      const Real V = (c.m1 * um1[q] + c.m2 * um2[q]) * c.inv_mc;
      const Real w = (um1[q] - um2[q]) * D;
      um1[q] = V + c.f1 * w;
      um2[q] = V - c.f2 * w;
    }
  }
  boris_rotate_kick(um1, c.a1, E1, B1, n1);
  boris_rotate_kick(um2, c.a2, E2, B2, n2);
}

// Reflecting walls `pad` cells inside non-periodic faces for a point
// particle (two-body ions: two_body_walls, per body).  off: new offset
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

// Decode the packed cell index (i | j << bx | k << (bx + by)).
template <int ND>
__device__ __forceinline__ void decode_cell(const GridInfo& g, uint32_t packed, int ci[3]) {
  ci[0] = packed & ((1u << g.bits[0]) - 1u);
  ci[1] = ND > 1 ? (packed >> g.bits[0]) & ((1u << g.bits[1]) - 1u) : 0;
  ci[2] = ND > 2 ? (packed >> (g.bits[0] + g.bits[1])) : 0;
}

template <int ND>
__device__ __forceinline__ uint32_t encode_cell(const GridInfo& g, const int cn[3]) {
  uint32_t pk = (uint32_t)cn[0];
  if (ND > 1) pk |= (uint32_t)cn[1] << g.bits[0];
  if (ND > 2) pk |= (uint32_t)cn[2] << (g.bits[0] + g.bits[1]);
  return pk;
}

// Sink for the general (four-node) deposit of one body, which a body
// needs only when its nearest node changes during the step.  The HBM
// kernels deposit at once (this sink takes nothing); the tiled kernel
// queues such bodies in LDS and deposits them after its particle loop, so
// that a wavefront does not run the long path for one or two lanes.
struct DepositNow {
  template <typename Real>
  __device__ __forceinline__ bool operator()(int, const Real*, const Real*, Real,
                                             const Real*) const {
    return false;
  }
};

// Stored state of one macro-particle: packed cell, offsets in the cell,
// momenta, relative displacement, per-particle omega_c and weight (when
// the species carries them).  Loaded ahead of its cycle so that the
// tiled kernel can fetch the next particle while advancing this one.
template <typename Real>
struct PState {
  uint32_t cell;
  Real off[3], u1[3], u2[3], dl[3], wc, w;
};

template <typename Real, int ND, bool TWO>
__device__ __forceinline__ void load_state(const SpeciesDev<Real>& s, const PushConst<Real>& c,
                                           int64_t p, PState<Real>& st) {
  st.cell = s.cell[p];
#pragma unroll
  for (int d = 0; d < 3; d++) st.off[d] = d < ND ? s.off[d][p] : Real(0);
#pragma unroll
  for (int q = 0; q < 3; q++) {
    st.u1[q] = s.u1[q][p];
    st.u2[q] = TWO ? s.u2[q][p] : Real(0);
    st.dl[q] = TWO ? s.dl[q][p] : Real(0);
  }
  st.wc = TWO && s.wc ? s.wc[p] : c.omega_c;
  st.w = s.w ? s.w[p] : Real(1);
}

// Along an axis with walls each body of an ion stays between the walls
// `pad` cells inside the faces (they mirror every body that reaches them),
// where every node its shape reaches is interior.  y: body positions
// relative to the cell ci.  A mirrored body's position is recomputed from
// the centre of mass and delta, so it can end a rounding error past the
// wall (a few units in the last place of the cell-relative position, some
// 1e-7 cell in FP32); the check allows kWallSlack cells for that (2^-16
// in FP32, 2^-40 in FP64), far less than moves any node of the shape.
template <typename Real>
struct WallSlack;
template <>
struct WallSlack<float> {
  static constexpr float value = 1.0f / 65536.0f;
};
template <>
struct WallSlack<double> {
  static constexpr double value = 1.0 / 1099511627776.0;  // 2^-40
};

template <typename Real, int ND>
__device__ __forceinline__ bool body_in_range(const GridInfo& g, const int ci[3],
                                              const Real y[3]) {
  constexpr Real kWallSlack = WallSlack<Real>::value;
  bool ok = true;
#pragma unroll
  for (int d = 0; d < ND; d++) {
    if (g.periodic[d]) continue;
    ok = ok && y[d] >= Real(g.pad - ci[d]) - kWallSlack &&
         y[d] <= Real(g.n[d] - g.pad - ci[d]) + kWallSlack;
  }
  return ok;
}

// Frame of a body at x (cell units, relative to the centre's cell ci): the
// cell that holds it (wrapped along periodic axes) as a storage index, and
// the offset there (x - floor(x), exact); k is the shift floor(x).
template <typename Real, int ND>
__device__ __forceinline__ int body_frame(const GridInfo& g, const int ci[3], const Real x[3],
                                          Real bx[3], int k[3]) {
  int64_t base = g.origin;
#pragma unroll
  for (int d = 0; d < 3; d++) {
    bx[d] = Real(0);
    k[d] = 0;
  }
#pragma unroll
  for (int d = 0; d < ND; d++) {
    const Real f = floor(x[d]);
    k[d] = static_cast<int>(f);
    bx[d] = x[d] - f;
    int b = ci[d] + k[d];
    if (g.periodic[d]) {
      b %= g.n[d];
      if (b < 0) b += g.n[d];
    }
    base += (int64_t)b * (d == 0 ? 1 : (d == 1 ? g.sy : g.sz));
  }
  return (int)base;
}

// One cycle of a two-body ion with a body outside [-1/2, 3/2) of its
// centre's cell along a resolved axis (Sec. 2: each body has its own
// position and momentum).  Each body is gathered and deposited from HBM in the frame of
// the cell that holds it (guard layers cover a window of any body in an
// interior cell; global atomics for the current); the centre of mass keeps
// the cell index, walls and crossing rule of the near path.  x1, x2: body
// positions relative to the centre's cell.
template <typename Real, int ND>
__device__ __forceinline__ void advance_far(const GridInfo& g, const SpeciesDev<Real>& s,
                                            const PushConst<Real>& c, int64_t p,
                                            const PState<Real>& st, const int ci[3],
                                            const Real x1[3], const Real x2[3],
                                            const FieldPtrs<Real>& f, uint32_t* err) {
  if (!body_in_range<Real, ND>(g, ci, x1) || !body_in_range<Real, ND>(g, ci, x2)) {
    atomicOr(err, PIC_ERR_RANGE);  // left untouched
    return;
  }
  const int sy = (int)g.sy, sz = (int)g.sz;
  Real b1[3], b2[3];
  int k1[3], k2[3], base1 = 0, base2 = 0;
  Real E1[3], B1[3], E2[3], B2[3];
  // one body at a time (loop not unrolled: one copy of the gather keeps
  // the registers low); results to their body by selects
#pragma unroll 1
  for (int body = 0; body < 2; body++) {
    Real xb[3], ob[3], Eb[3], Bb[3];
    int kk[3];
#pragma unroll
    for (int d = 0; d < 3; d++) xb[d] = body == 0 ? x1[d] : x2[d];
    const int bs = body_frame<Real, ND>(g, ci, xb, ob, kk);
    gather<Real, ND>(f, bs, sy, sz, ob, Eb, Bb);
    base1 = body == 0 ? bs : base1;
    base2 = body == 0 ? base2 : bs;
#pragma unroll
    for (int q = 0; q < 3; q++) {
      b1[q] = body == 0 ? ob[q] : b1[q];
      b2[q] = body == 0 ? b2[q] : ob[q];
      k1[q] = body == 0 ? kk[q] : k1[q];
      k2[q] = body == 0 ? k2[q] : kk[q];
      E1[q] = body == 0 ? Eb[q] : E1[q];
      B1[q] = body == 0 ? Bb[q] : B1[q];
      E2[q] = body == 0 ? E2[q] : Eb[q];
      B2[q] = body == 0 ? B2[q] : Bb[q];
    }
  }
  Real u1[3], u2[3], dl[3], off[3] = {0, 0, 0};
#pragma unroll
  for (int q = 0; q < 3; q++) {
    u1[q] = st.u1[q];
    u2[q] = st.u2[q];
    dl[q] = st.dl[q];
  }
#pragma unroll
  for (int d = 0; d < ND; d++) off[d] = st.off[d];
  const Real wc = st.wc;
  Real n1[3], n2[3];
  two_body_kick(c, wc, ion_inv_ac2(c, s.wc != nullptr, wc), dl, u1, u2, E1, B1, E2, B2, n1, n2);
  const Real ig1 = rsqrt1(Real(1) + n1[0] * n1[0] + n1[1] * n1[1] + n1[2] * n1[2]);
  const Real ig2 = rsqrt1(Real(1) + n2[0] * n2[0] + n2[1] * n2[1] + n2[2] * n2[2]);
  Real v1[3], v2[3];
#pragma unroll
  for (int q = 0; q < 3; q++) {
    v1[q] = n1[q] * ig1;
    v2[q] = n2[q] * ig2;
    dl[q] = dl[q] + c.dt * (v1[q] - v2[q]);
  }
  Real offn[3] = {0, 0, 0};
#pragma unroll
  for (int d = 0; d < ND; d++)
    offn[d] = off[d] + c.dt * (c.m1 * v1[d] + c.m2 * v2[d]) * c.inv_mc * c.idx[d];
  two_body_walls<Real, ND>(g, c, ci, offn, dl, n1, n2);
  Real y1[3] = {0, 0, 0}, y2[3] = {0, 0, 0};
#pragma unroll
  for (int d = 0; d < ND; d++) {
    const Real sd = dl[d] * c.idx[d];
    y1[d] = offn[d] + c.f1 * sd;
    y2[d] = offn[d] - c.f2 * sd;
  }
  bool range_ok = body_in_range<Real, ND>(g, ci, y1) && body_in_range<Real, ND>(g, ci, y2);
  if (c.deposit) {
    const Real W = st.w;
    const Real qw1 = s.w ? c.q1 * W : c.qw1;
    const Real qw2 = s.w ? c.q2 * W : c.qw2;
    // new positions in each body's old frame
    Real z1[3] = {0, 0, 0}, z2[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < ND; d++) {
      z1[d] = y1[d] - Real(k1[d]);
      z2[d] = y2[d] - Real(k2[d]);
    }
    // displacements from the stored quantities, as in the near path
    Real d1[3] = {0, 0, 0}, d2[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < ND; d++) {
      const Real dR = offn[d] - off[d];
      const Real dd = (dl[d] - st.dl[d]) * c.idx[d];
      d1[d] = dR + c.f1 * dd;
      d2[d] = dR - c.f2 * dd;
    }
    Real* const J[3] = {f.J[0], f.J[1], f.J[2]};
#pragma unroll 1
    for (int body = 0; body < 2; body++) {
      Real ob[3], zb[3], vb[3], db[3];
#pragma unroll
      for (int q = 0; q < 3; q++) {
        ob[q] = body == 0 ? b1[q] : b2[q];
        zb[q] = body == 0 ? z1[q] : z2[q];
        vb[q] = body == 0 ? v1[q] : v2[q];
        db[q] = body == 0 ? d1[q] : d2[q];
      }
      const int bb = body == 0 ? base1 : base2;
      const Real qb = body == 0 ? qw1 : qw2;
      const Real* xs[2] = {ob, zb};
      int nn[3];
      // a body that keeps its nearest node: the three-node window
      if (common_node<Real, ND>(xs, 2, nn))
        deposit3<Real, ND, true, Real, false>(J, bb, sy, sz, nn, ob, db, qb, vb, ob, db, Real(0),
                                              vb, c);
      else
        range_ok = deposit<Real, ND, true, Real>(J, bb, sy, sz, ob, zb, qb, vb, c) && range_ok;
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
  if (!(finite3(n1) && finite3(n2) && finite3(dl))) atomicOr(err, PIC_ERR_NAN);
  s.cell[p] = encode_cell<ND>(g, cn);
#pragma unroll
  for (int d = 0; d < ND; d++) s.off[d][p] = offn[d];
#pragma unroll
  for (int q = 0; q < 3; q++) {
    s.u1[q][p] = n1[q];
    s.u2[q][p] = n2[q];
    s.dl[q][p] = dl[q];
  }
}

// Advance macro-particle p through one full cycle.  Gather reads E, B
// through `fg` at index `fbase` of the particle's cell (strides fsy, fsz);
// the deposit adds into J at `jbase` (strides jsy, jsz).  GLOBAL selects
// the HBM form of the deposit (atomics, zero terms skipped).  `later`
// may take over a body's general deposit (returns true if it did).
template <typename Real, int ND, bool TWO, bool GLOBAL, typename JT = Real,
          typename Later = DepositNow>
__device__ __forceinline__ void advance_particle(const GridInfo& g, const SpeciesDev<Real>& s,
                                                 const PushConst<Real>& c, int64_t p,
                                                 const PState<Real>& st, const int ci[3],
                                                 const FieldPtrs<Real>& fg, int fbase, int fsy,
                                                 int fsz, JT* const J[3], int jbase, int jsy,
                                                 int jsz, uint32_t* err,
                                                 const Later& later = Later{}) {
  Real off[3] = {0, 0, 0};
#pragma unroll
  for (int d = 0; d < ND; d++) off[d] = st.off[d];
  Real u1[3], u2[3] = {0, 0, 0}, dl[3] = {0, 0, 0};
#pragma unroll
  for (int q = 0; q < 3; q++) u1[q] = st.u1[q];
  if constexpr (TWO) {
#pragma unroll
    for (int q = 0; q < 3; q++) {
      u2[q] = st.u2[q];
      dl[q] = st.dl[q];
    }
  }
  const Real W = st.w;

  // body positions (cell units, relative to the cell)
  Real x1[3] = {0, 0, 0}, x2[3] = {0, 0, 0};
  bool finite = finite3(u1) && finite3(u2) && finite3(dl);
  bool inside = true, near = true;
#pragma unroll
  for (int d = 0; d < ND; d++) {
    finite = finite && isfinite(off[d]);
    inside = inside && (off[d] >= Real(0)) && (off[d] <= Real(1));
    if constexpr (TWO) {
      Real sd = dl[d] * c.idx[d];
      x1[d] = off[d] + c.f1 * sd;
      x2[d] = off[d] - c.f2 * sd;
      near = near && body_near(x1[d]) && body_near(x2[d]);
    } else {
      x1[d] = off[d];
    }
  }
  if (!finite || !inside) {
    // a particle that cannot be gathered safely is left untouched
    atomicOr(err, finite ? PIC_ERR_RANGE : PIC_ERR_NAN);
    return;
  }
  if constexpr (TWO) {
    if (!near) {
      // a body beyond the reach of the cell frame: each body in its own
      // cell frame, from HBM (the tiled kernel lists such ions for the HBM
      // pass)
      if constexpr (GLOBAL)
        advance_far<Real, ND>(g, s, c, p, st, ci, x1, x2, fg, err);
      else
        atomicOr(err, PIC_ERR_RANGE);
      return;
    }
  }

  if constexpr (TWO) {
    const Real wc = st.wc;
    // one body at a time (loop not unrolled: a single copy of the gather
    // keeps the live register set small); E and B are kept per body for
    // the second half kick
    Real E1[3], B1[3], E2[3], B2[3];
    if (same_stencil<Real, ND>(x1, x2)) {
      // both bodies on the same nodes (the usual case: |delta| << dx)
      gather2<Real, ND>(fg, fbase, fsy, fsz, x1, x2, E1, B1, E2, B2);
    } else {
#pragma unroll 1
    for (int body = 0; body < 2; body++) {
      Real xb[3], Eb[3], Bb[3];
#pragma unroll
      for (int d = 0; d < 3; d++) xb[d] = body == 0 ? x1[d] : x2[d];
      gather<Real, ND>(fg, fbase, fsy, fsz, xb, Eb, Bb);
#pragma unroll
      for (int q = 0; q < 3; q++) {
        E1[q] = body == 0 ? Eb[q] : E1[q];
        B1[q] = body == 0 ? Bb[q] : B1[q];
        E2[q] = body == 0 ? E2[q] : Eb[q];
        B2[q] = body == 0 ? B2[q] : Bb[q];
      }
    }
    }
    Real n1[3], n2[3];
    two_body_kick(c, wc, ion_inv_ac2(c, s.wc != nullptr, wc), dl, u1, u2, E1, B1, E2, B2, n1,
                  n2);
    Real ig1 = rsqrt1(Real(1) + n1[0] * n1[0] + n1[1] * n1[1] + n1[2] * n1[2]);
    Real ig2 = rsqrt1(Real(1) + n2[0] * n2[0] + n2[1] * n2[1] + n2[2] * n2[2]);
    Real v1[3], v2[3];
#pragma unroll
    for (int q = 0; q < 3; q++) {
      v1[q] = n1[q] * ig1;
      v2[q] = n2[q] * ig2;
      dl[q] = dl[q] + c.dt * (v1[q] - v2[q]);
    }
    // move: R += dt (m1 v1 + m2 v2)/m_c, delta += dt (v1 - v2); walls per body
    Real offn[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < ND; d++)
      offn[d] = off[d] + c.dt * (c.m1 * v1[d] + c.m2 * v2[d]) * c.inv_mc * c.idx[d];
    two_body_walls<Real, ND>(g, c, ci, offn, dl, n1, n2);
    Real y1[3] = {0, 0, 0}, y2[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < ND; d++) {
      Real sd = dl[d] * c.idx[d];
      y1[d] = offn[d] + c.f1 * sd;
      y2[d] = offn[d] - c.f2 * sd;
    }
    // along walled axes the bodies stay between the walls
    bool range_ok = body_in_range<Real, ND>(g, ci, y1) && body_in_range<Real, ND>(g, ci, y2);
    if (c.deposit) {
      const Real qw1 = s.w ? c.q1 * W : c.qw1;
      const Real qw2 = s.w ? c.q2 * W : c.qw2;
      const Real* xs[4] = {x1, x2, y1, y2};
      int nn[3];
      const bool pair = common_node<Real, ND>(xs, 4, nn);
      if (pair) {
        // both bodies keep one nearest node: merged three-node deposit.
        // Displacements from the stored quantities (centre-of-mass offset,
        // delta), whose differences over a step are exact in the working
        // precision, not from the rounded body positions.
        Real d1[3] = {0, 0, 0}, d2[3] = {0, 0, 0};
#pragma unroll
        for (int d = 0; d < ND; d++) {
          const Real dR = offn[d] - off[d];
          const Real dd = (dl[d] - st.dl[d]) * c.idx[d];
          d1[d] = dR + c.f1 * dd;
          d2[d] = dR - c.f2 * dd;
        }
        deposit3<Real, ND, GLOBAL, JT, true>(J, jbase, jsy, jsz, nn, x1, d1, qw1, v1, x2, d2,
                                             qw2, v2, c);
      } else {
#pragma unroll 1
      for (int body = 0; body < 2; body++) {
        Real xa[3], y[3] = {0, 0, 0}, vb[3];
#pragma unroll
        for (int d = 0; d < 3; d++) {
          xa[d] = body == 0 ? x1[d] : x2[d];
          vb[d] = body == 0 ? v1[d] : v2[d];
        }
#pragma unroll
        for (int d = 0; d < ND; d++) {
          Real sd = dl[d] * c.idx[d];
          y[d] = body == 0 ? offn[d] + c.f1 * sd : offn[d] - c.f2 * sd;
        }
        const Real qb = body == 0 ? qw1 : qw2;
        const Real* xb2[2] = {xa, y};
        int nb[3];
        // FP32: a body that keeps its nearest node takes its own three-node
        // window, with the displacement from the stored quantities (the
        // FP64 tiled build measured more instructions per particle with
        // this branch, and keeps the general window)
        if (sizeof(Real) == 4 && common_node<Real, ND>(xb2, 2, nb)) {
          Real db[3] = {0, 0, 0};
#pragma unroll
          for (int d = 0; d < ND; d++) {
            const Real dR = offn[d] - off[d];
            const Real dd = (dl[d] - st.dl[d]) * c.idx[d];
            db[d] = body == 0 ? dR + c.f1 * dd : dR - c.f2 * dd;
          }
          deposit3<Real, ND, GLOBAL, JT, false>(J, jbase, jsy, jsz, nb, xa, db, qb, vb, xa, db,
                                                Real(0), vb, c);
        } else if (!later(jbase, xa, y, qb, vb)) {
          range_ok = deposit<Real, ND, GLOBAL, JT>(J, jbase, jsy, jsz, xa, y, qb, vb, c) && range_ok;
        }
      }
      }
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
    s.cell[p] = encode_cell<ND>(g, cn);
#pragma unroll
    for (int d = 0; d < ND; d++) s.off[d][p] = offn[d];
#pragma unroll
    for (int q = 0; q < 3; q++) {
      s.u1[q][p] = n1[q];
      s.u2[q][p] = n2[q];
      s.dl[q][p] = dl[q];
    }
  } else {
    Real E1[3], B1[3];
    gather<Real, ND>(fg, fbase, fsy, fsz, x1, E1, B1);
    Real um[3], n1[3], v1[3];
#pragma unroll
    for (int q = 0; q < 3; q++) um[q] = u1[q] + c.a1 * E1[q];
    boris_rotate_kick(um, c.a1, E1, B1, n1);
    Real ig = rsqrt1(Real(1) + n1[0] * n1[0] + n1[1] * n1[1] + n1[2] * n1[2]);
#pragma unroll
    for (int q = 0; q < 3; q++) v1[q] = n1[q] * ig;
    Real y1[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < ND; d++) {
      y1[d] = off[d] + c.dt * v1[d] * c.idx[d];
      if (reflect(g.periodic[d], ci[d], g.n[d], g.pad, y1[d])) n1[d] = -n1[d];
    }
    bool range_ok = true;
    if (c.deposit) {
      const Real qw1 = s.w ? c.q1 * W : c.qw1;
      const Real* xs[2] = {x1, y1};
      int nn[3];
      const bool keep = common_node<Real, ND>(xs, 2, nn);
      // per lane: most particles keep their nearest node
      if (keep) {
        Real d1[3] = {0, 0, 0};
#pragma unroll
        for (int d = 0; d < ND; d++) d1[d] = y1[d] - x1[d];
        deposit3<Real, ND, GLOBAL, JT, false>(J, jbase, jsy, jsz, nn, x1, d1, qw1, v1, x1, d1,
                                              Real(0), v1, c);
      }
      else if (!later(jbase, x1, y1, qw1, v1))
        range_ok = deposit<Real, ND, GLOBAL, JT>(J, jbase, jsy, jsz, x1, y1, qw1, v1, c);
    }
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
    s.cell[p] = encode_cell<ND>(g, cn);
#pragma unroll
    for (int d = 0; d < ND; d++) s.off[d][p] = y1[d];
#pragma unroll
    for (int q = 0; q < 3; q++) s.u1[q][p] = n1[q];
  }
}

}  // namespace pic
