// adjoint.hip -- reverse-mode (adjoint) particle cycle of the gradient run,
// 1D, 2D and 3D grids, two-body ions and point particles.
//
// One thread per macro-particle (one workgroup per tile of the sorted order
// when the tile offsets are given).  The thread recomputes the forward cycle
// of its particle from the stored state at the start of the step (the
// same arithmetic as the forward kernels: quadratic B-spline gather,
// softened bond force, time-centred friction, relativistic Boris push of
// each body, move, walls, Esirkepov deposit; Sec. 2 and Sec. 3.1) and then
// applies its transpose:
//   * the deposit's adjoint reads the adjoint current lJ on the deposit
//     window and yields derivatives with respect to the old and new body
//     positions (through the B-spline weights and their derivatives) and
//     to the out-of-plane velocity;
//   * move, Lorentz factor, Boris rotation, friction and kicks are
//     differentiated in reverse order;
//   * the gather's adjoint scatters lambda_E, lambda_B of each body onto the
//     nodes with the gather weights (into an FP64 LDS patch of the tile, or
//     with atomics into lE, lB) and adds the position derivative of the
//     interpolant.
// The particle's adjoint state (offsets, delta, u1, u2) is updated in
// place; the derivatives with respect to omega_c and the friction rate are
// reduced per block and added to two FP64 accumulators.
#include "adjoint.h"

namespace pic {

namespace {

// Component planes of a field array stored contiguously (E0..E2, B0..B2,
// J0..J2, `plane` values apart): one base pointer instead of nine keeps
// the kernel arguments in few scalar registers.
template <typename Real>
struct Planes {
  Real* base;
  int64_t plane;
  __device__ __forceinline__ Real* E(int a) const { return base + a * plane; }
  __device__ __forceinline__ Real* B(int a) const { return base + (3 + a) * plane; }
  __device__ __forceinline__ Real* J(int a) const { return base + (6 + a) * plane; }
};

// Quadratic B-spline weights and their derivatives with respect to the
// position at the nearest node n = floor(x + 1/2) (integer stagger) or
// n = floor(x) (half stagger, node i at i + 1/2): nodes n-1, n, n+1.
template <typename Real>
struct Shape {
  int i0;  // first node relative to the cell
  Real w[3], dw[3];
};

template <typename Real>
__device__ __forceinline__ Shape<Real> shape_at(Real x, bool half) {
  Shape<Real> s;
  const Real f = half ? floor(x) : floor(x + Real(0.5));
  const Real d = half ? x - f - Real(0.5) : x - f;
  const Real a = Real(0.5) - d, b = Real(0.5) + d;
  s.i0 = static_cast<int>(f) - 1;
  s.w[0] = Real(0.5) * a * a;
  s.w[1] = Real(0.75) - d * d;
  s.w[2] = Real(0.5) * b * b;
  s.dw[0] = -a;
  s.dw[1] = Real(-2) * d;
  s.dw[2] = b;
  return s;
}

template <typename Real>
__device__ __forceinline__ Shape<Real> unit_shape() {
  Shape<Real> s;
  s.i0 = 0;
  s.w[0] = Real(1);
  s.w[1] = s.w[2] = Real(0);
  s.dw[0] = s.dw[1] = s.dw[2] = Real(0);
  return s;
}

// Destination of the gather's transpose for one particle: an FP64 LDS
// patch of the workgroup's tile (component planes of `lplane` values,
// strides lsy, lsz, the particle's cell at index `lbase`), or the global
// adjoint planes with atomics (particles outside their tile).  Nodes are
// given relative to the particle's cell.
template <typename Real>
struct Sink {
  Planes<Real> l;
  int gbase, gsy, gsz;  // 32-bit: a plane holds fewer than 2^31 values
  double* lds;
  int lbase, lsy, lsz, lplane;
  __device__ __forceinline__ void add(int comp, int ix, int iy, int iz, Real v) const {
    if (lds) {
      atomicAdd(lds + comp * lplane + lbase + ix + iy * lsy + iz * lsz, (double)v);
    } else {
      Real* F = l.base + comp * l.plane;
      unsafeAtomicAdd(F + gbase + ix + iy * gsy + iz * gsz, v);
    }
  }
};

// Quadratic B-spline shapes of one body at the integer (n) and half (h)
// staggers of each resolved axis (unit shapes along unresolved ones).
template <typename Real>
struct Stencil {
  Shape<Real> n[3], h[3];
};

template <typename Real, int ND>
__device__ __forceinline__ Stencil<Real> stencil_at(const Real x[3]) {
  Stencil<Real> s;
#pragma unroll
  for (int d = 0; d < 3; d++) {
    if (d < ND) {
      s.n[d] = shape_at(x[d], false);
      s.h[d] = shape_at(x[d], true);
    } else {
      s.n[d] = s.h[d] = unit_shape<Real>();
    }
  }
  return s;
}

// Node offsets and strides of one interpolation: the base index of the
// particle's cell and the y, z strides of the array read.
struct Where3 {
  int base, sy, sz;  // 32-bit: a plane holds fewer than 2^31 values
};

template <typename Real, int ND>
__device__ __forceinline__ Real interp_value(const Real* __restrict__ F, const Where3& w,
                                             const Shape<Real>& sx, const Shape<Real>& syy,
                                             const Shape<Real>& szz) {
  Real v = 0;
  constexpr int NY = ND > 1 ? 3 : 1, NZ = ND > 2 ? 3 : 1;
#pragma unroll
  for (int t = 0; t < NZ; t++) {
    Real vy = 0;
#pragma unroll
    for (int s = 0; s < NY; s++) {
      const Real* row = F + (w.base + sx.i0 + (ND > 1 ? (syy.i0 + s) * w.sy : 0) +
                             (ND > 2 ? (szz.i0 + t) * w.sz : 0));
      const Real wy = ND > 1 ? syy.w[s] : Real(1);
      vy += wy * (sx.w[0] * row[0] + sx.w[1] * row[1] + sx.w[2] * row[2]);
    }
    v += (ND > 2 ? szz.w[t] : Real(1)) * vy;
  }
  return v;
}

// E and B at a body position (the gather of the forward cycle): E_a
// half-staggered along a, B_a along the two other axes.
template <typename Real, int ND>
__device__ __forceinline__ void gather_values(const Planes<Real>& f, const Where3& w,
                                              const Real x[3], Real E[3], Real B[3]) {
  const Stencil<Real> t = stencil_at<Real, ND>(x);
  E[0] = interp_value<Real, ND>(f.E(0), w, t.h[0], t.n[1], t.n[2]);
  E[1] = interp_value<Real, ND>(f.E(1), w, t.n[0], t.h[1], t.n[2]);
  E[2] = interp_value<Real, ND>(f.E(2), w, t.n[0], t.n[1], t.h[2]);
  B[0] = interp_value<Real, ND>(f.B(0), w, t.n[0], t.h[1], t.h[2]);
  B[1] = interp_value<Real, ND>(f.B(1), w, t.h[0], t.n[1], t.h[2]);
  B[2] = interp_value<Real, ND>(f.B(2), w, t.h[0], t.h[1], t.n[2]);
}

// True when two bodies' stencils start at the same nodes for every stagger.
template <typename Real, int ND>
__device__ __forceinline__ bool same_nodes(const Stencil<Real>& a, const Stencil<Real>& b) {
  bool same = true;
#pragma unroll
  for (int d = 0; d < ND; d++) same = same && a.n[d].i0 == b.n[d].i0 && a.h[d].i0 == b.h[d].i0;
  return same;
}

// Two bodies whose stencils share the nodes: one pass over the nodes
// interpolates both.
template <typename Real, int ND>
__device__ __forceinline__ void interp_value2(const Real* __restrict__ F, const Where3& w,
                                              const Shape<Real>& ax, const Shape<Real>& ay,
                                              const Shape<Real>& az, const Shape<Real>& bx,
                                              const Shape<Real>& by, const Shape<Real>& bz,
                                              Real& va, Real& vb) {
  va = vb = Real(0);
  constexpr int NY = ND > 1 ? 3 : 1, NZ = ND > 2 ? 3 : 1;
#pragma unroll
  for (int t = 0; t < NZ; t++) {
    Real ya = 0, yb = 0;
#pragma unroll
    for (int s = 0; s < NY; s++) {
      const Real* row = F + (w.base + ax.i0 + (ND > 1 ? (ay.i0 + s) * w.sy : 0) +
                             (ND > 2 ? (az.i0 + t) * w.sz : 0));
      const Real r0 = row[0], r1 = row[1], r2 = row[2];
      ya += (ND > 1 ? ay.w[s] : Real(1)) * (ax.w[0] * r0 + ax.w[1] * r1 + ax.w[2] * r2);
      yb += (ND > 1 ? by.w[s] : Real(1)) * (bx.w[0] * r0 + bx.w[1] * r1 + bx.w[2] * r2);
    }
    va += (ND > 2 ? az.w[t] : Real(1)) * ya;
    vb += (ND > 2 ? bz.w[t] : Real(1)) * yb;
  }
}

// E and B at both body positions of an ion (shared node reads when their
// stencils coincide).
template <typename Real, int ND>
__device__ __forceinline__ void gather_values2(const Planes<Real>& f, const Where3& w,
                                               const Real x1[3], const Real x2[3], Real E1[3],
                                               Real B1[3], Real E2[3], Real B2[3]) {
  const Stencil<Real> a = stencil_at<Real, ND>(x1), b = stencil_at<Real, ND>(x2);
  if (same_nodes<Real, ND>(a, b)) {
    interp_value2<Real, ND>(f.E(0), w, a.h[0], a.n[1], a.n[2], b.h[0], b.n[1], b.n[2], E1[0], E2[0]);
    interp_value2<Real, ND>(f.E(1), w, a.n[0], a.h[1], a.n[2], b.n[0], b.h[1], b.n[2], E1[1], E2[1]);
    interp_value2<Real, ND>(f.E(2), w, a.n[0], a.n[1], a.h[2], b.n[0], b.n[1], b.h[2], E1[2], E2[2]);
    interp_value2<Real, ND>(f.B(0), w, a.n[0], a.h[1], a.h[2], b.n[0], b.h[1], b.h[2], B1[0], B2[0]);
    interp_value2<Real, ND>(f.B(1), w, a.h[0], a.n[1], a.h[2], b.h[0], b.n[1], b.h[2], B1[1], B2[1]);
    interp_value2<Real, ND>(f.B(2), w, a.h[0], a.h[1], a.n[2], b.h[0], b.h[1], b.n[2], B1[2], B2[2]);
  } else {
    gather_values<Real, ND>(f, w, x1, E1, B1);
    gather_values<Real, ND>(f, w, x2, E2, B2);
  }
}

// Adjoint of one interpolated component for one body (or, with two shapes,
// for both bodies of an ion whose stencils share the nodes), in one pass
// over its nodes: scatter lam * weight(node) and add lam * d(interp)/dx
// to lx.
template <typename Real, int ND, bool PAIR>
__device__ __forceinline__ void comp_adjoint(const Real* __restrict__ F, int comp,
                                             const Sink<Real>& k, const Where3& w,
                                             const Shape<Real>& ax, const Shape<Real>& ay,
                                             const Shape<Real>& az, Real la,
                                             const Shape<Real>& bx, const Shape<Real>& by,
                                             const Shape<Real>& bz, Real lb, Real lxa[3],
                                             Real lxb[3]) {
  if (la == Real(0) && (!PAIR || lb == Real(0))) return;
  constexpr int NY = ND > 1 ? 3 : 1, NZ = ND > 2 ? 3 : 1;
#pragma unroll
  for (int t = 0; t < NZ; t++) {
    const int iz = ND > 2 ? az.i0 + t : 0;
#pragma unroll
    for (int s = 0; s < NY; s++) {
      const int iy = ND > 1 ? ay.i0 + s : 0;
      const Real* row = F + (w.base + ax.i0 + (ND > 1 ? iy * w.sy : 0) + (ND > 2 ? iz * w.sz : 0));
      const Real r0 = row[0], r1 = row[1], r2 = row[2];
      const Real wza = ND > 2 ? az.w[t] : Real(1), wya = ND > 1 ? ay.w[s] : Real(1);
      const Real va = ax.w[0] * r0 + ax.w[1] * r1 + ax.w[2] * r2;
      lxa[0] += la * wza * wya * (ax.dw[0] * r0 + ax.dw[1] * r1 + ax.dw[2] * r2);
      if (ND > 1) lxa[1] += la * wza * ay.dw[s] * va;
      if (ND > 2) lxa[2] += la * az.dw[t] * wya * va;
      const Real ca = la * wza * wya;
      Real cb = 0;
      if constexpr (PAIR) {
        const Real wzb = ND > 2 ? bz.w[t] : Real(1), wyb = ND > 1 ? by.w[s] : Real(1);
        const Real vb = bx.w[0] * r0 + bx.w[1] * r1 + bx.w[2] * r2;
        lxb[0] += lb * wzb * wyb * (bx.dw[0] * r0 + bx.dw[1] * r1 + bx.dw[2] * r2);
        if (ND > 1) lxb[1] += lb * wzb * by.dw[s] * vb;
        if (ND > 2) lxb[2] += lb * bz.dw[t] * wyb * vb;
        cb = lb * wzb * wyb;
      }
#pragma unroll
      for (int r = 0; r < 3; r++)
        k.add(comp, ax.i0 + r, iy, iz, PAIR ? ca * ax.w[r] + cb * bx.w[r] : ca * ax.w[r]);
    }
  }
}

// The gather's transpose for one body, or for both bodies of an ion whose
// stencils share the nodes (PAIR).
template <typename Real, int ND, bool PAIR>
__device__ __forceinline__ void gather_adjoint(const Planes<Real>& f, const Sink<Real>& k,
                                               const Where3& w, const Stencil<Real>& a,
                                               const Real lEa[3], const Real lBa[3],
                                               const Stencil<Real>& b, const Real lEb[3],
                                               const Real lBb[3], Real lxa[3], Real lxb[3]) {
  comp_adjoint<Real, ND, PAIR>(f.E(0), 0, k, w, a.h[0], a.n[1], a.n[2], lEa[0], b.h[0], b.n[1], b.n[2], lEb[0], lxa, lxb);
  comp_adjoint<Real, ND, PAIR>(f.E(1), 1, k, w, a.n[0], a.h[1], a.n[2], lEa[1], b.n[0], b.h[1], b.n[2], lEb[1], lxa, lxb);
  comp_adjoint<Real, ND, PAIR>(f.E(2), 2, k, w, a.n[0], a.n[1], a.h[2], lEa[2], b.n[0], b.n[1], b.h[2], lEb[2], lxa, lxb);
  comp_adjoint<Real, ND, PAIR>(f.B(0), 3, k, w, a.n[0], a.h[1], a.h[2], lBa[0], b.n[0], b.h[1], b.h[2], lBb[0], lxa, lxb);
  comp_adjoint<Real, ND, PAIR>(f.B(1), 4, k, w, a.h[0], a.n[1], a.h[2], lBa[1], b.h[0], b.n[1], b.h[2], lBb[1], lxa, lxb);
  comp_adjoint<Real, ND, PAIR>(f.B(2), 5, k, w, a.h[0], a.h[1], a.n[2], lBa[2], b.h[0], b.h[1], b.n[2], lBb[2], lxa, lxb);
}


__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }

template <typename Real>
__device__ __forceinline__ void cross(const Real a[3], const Real b[3], Real c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// Boris rotation and second half kick: out = um + (um + um x t) x s + a E,
// t = a B / gamma(um), s = 2 t / (1 + t^2).  Reverse mode: given lout,
// adds to lum, lE, lB.
template <typename Real>
__device__ __forceinline__ void boris_forward(const Real um[3], Real a, const Real E[3],
                                              const Real B[3], Real out[3]) {
  const Real g = rsq(Real(1) + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
  const Real k = a * g;
  Real t[3] = {k * B[0], k * B[1], k * B[2]};
  const Real sk = Real(2) * rcp(Real(1) + t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
  Real s[3] = {sk * t[0], sk * t[1], sk * t[2]};
  Real c[3], w[3], ws[3];
  cross(um, t, c);
#pragma unroll
  for (int q = 0; q < 3; q++) w[q] = um[q] + c[q];
  cross(w, s, ws);
#pragma unroll
  for (int q = 0; q < 3; q++) out[q] = um[q] + ws[q] + a * E[q];
}

template <typename Real>
__device__ __forceinline__ void boris_adjoint(const Real um[3], Real a, const Real B[3],
                                              const Real lout[3], Real lum[3], Real lE[3],
                                              Real lB[3]) {
  const Real g = rsq(Real(1) + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
  const Real k = a * g;
  Real t[3] = {k * B[0], k * B[1], k * B[2]};
  const Real sk = Real(2) * rcp(Real(1) + t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
  Real s[3] = {sk * t[0], sk * t[1], sk * t[2]};
  Real c[3], w[3];
  cross(um, t, c);
#pragma unroll
  for (int q = 0; q < 3; q++) w[q] = um[q] + c[q];
  // out = um + w x s + a E
  Real lw[3], ls[3], lt[3], tmp[3];
  cross(s, lout, lw);   // lambda . (w x s) = w . (s x lambda)
  cross(lout, w, ls);   //                 = s . (lambda x w)
#pragma unroll
  for (int q = 0; q < 3; q++) {
    lum[q] += lout[q] + lw[q];
    lE[q] += a * lout[q];
  }
  // w = um + um x t
  cross(t, lw, tmp);
#pragma unroll
  for (int q = 0; q < 3; q++) lum[q] += tmp[q];
  cross(lw, um, lt);
  // s = sk t, sk = 2 / (1 + t.t)
  const Real lsk = t[0] * ls[0] + t[1] * ls[1] + t[2] * ls[2];
  const Real ltt = -Real(0.5) * sk * sk * lsk;
#pragma unroll
  for (int q = 0; q < 3; q++) lt[q] += sk * ls[q] + Real(2) * t[q] * ltt;
  // t = a g B
  Real lk = 0;
#pragma unroll
  for (int q = 0; q < 3; q++) {
    lB[q] += k * lt[q];
    lk += B[q] * lt[q];
  }
  const Real lg = a * lk;
  const Real g3 = g * g * g;
#pragma unroll
  for (int q = 0; q < 3; q++) lum[q] -= g3 * um[q] * lg;
}

// v = n / sqrt(1 + n^2): lambda_n += g lv - g^3 n (n . lv)
template <typename Real>
__device__ __forceinline__ void velocity_adjoint(const Real n[3], const Real lv[3], Real ln[3]) {
  const Real g = rsq(Real(1) + n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  const Real nl = n[0] * lv[0] + n[1] * lv[1] + n[2] * lv[2];
  const Real g3 = g * g * g;
#pragma unroll
  for (int q = 0; q < 3; q++) ln[q] += g * lv[q] - g3 * n[q] * nl;
}

// Shapes of one body on the deposit window of one dimension, NW nodes
// from node `lo`: old (S0) and new (S1) weights and their position
// derivatives.  NW = 3 when the body keeps its nearest node over the step
// (the window of its shape), NW = 4 when that node moves by one.
template <typename Real, int NW>
struct Win {
  int lo;
  Real S0[NW], S1[NW], D0[NW], D1[NW];
};

template <typename Real>
__device__ __forceinline__ bool win_build(Real x0, Real x1, Win<Real, 3>& w) {
  const Shape<Real> a = shape_at(x0, false), b = shape_at(x1, false);
  if (a.i0 != b.i0) return false;
  w.lo = a.i0;
#pragma unroll
  for (int r = 0; r < 3; r++) {
    w.S0[r] = a.w[r];
    w.D0[r] = a.dw[r];
    w.S1[r] = b.w[r];
    w.D1[r] = b.dw[r];
  }
  return true;
}

template <typename Real>
__device__ __forceinline__ bool win_build(Real x0, Real x1, Win<Real, 4>& w) {
  const Shape<Real> a = shape_at(x0, false), b = shape_at(x1, false);
  const int lo = min(a.i0, b.i0);
  const int sa = a.i0 - lo, sb = b.i0 - lo;
  if (sa > 1 || sb > 1) return false;
  w.lo = lo;
  // the three weights sit at window nodes sa..sa+2 (sa = 0 or 1); selects,
  // not a runtime index, keep them in registers
  w.S0[0] = sa ? Real(0) : a.w[0];
  w.S0[1] = sa ? a.w[0] : a.w[1];
  w.S0[2] = sa ? a.w[1] : a.w[2];
  w.S0[3] = sa ? a.w[2] : Real(0);
  w.D0[0] = sa ? Real(0) : a.dw[0];
  w.D0[1] = sa ? a.dw[0] : a.dw[1];
  w.D0[2] = sa ? a.dw[1] : a.dw[2];
  w.D0[3] = sa ? a.dw[2] : Real(0);
  w.S1[0] = sb ? Real(0) : b.w[0];
  w.S1[1] = sb ? b.w[0] : b.w[1];
  w.S1[2] = sb ? b.w[1] : b.w[2];
  w.S1[3] = sb ? b.w[2] : Real(0);
  w.D1[0] = sb ? Real(0) : b.dw[0];
  w.D1[1] = sb ? b.dw[0] : b.dw[1];
  w.D1[2] = sb ? b.dw[1] : b.dw[2];
  w.D1[3] = sb ? b.dw[2] : Real(0);
  return true;
}

// Adjoint of the Esirkepov deposit of NB bodies on common windows (which
// then read the adjoint current once; the kernels call it one body at a
// time, which keeps their registers within two waves per SIMD), body
// b with charge Q[b] moving from x0[b] to x1[b] at velocity v[b] (for the
// out-of-plane components), on windows of NW nodes: with lJ the adjoint
// current, Phi = sum lJ . J; returns per body dPhi/dx0, dPhi/dx1 (resolved
// dims) and dPhi/dv (unresolved components).  The running sum along an
// axis (non-zero on the first NW - 1 edges of the window: the shape change
// sums to zero) turns into a suffix sum of lJ; the path-averaged
// transverse shape M = S0 S0'/3 + S0 S1'/6 + S1 S0'/6 + S1 S1'/3 (two
// transverse axes) or (S0 + S1)/2 (one) is differentiated by hand.
// Returns false if the windows do not hold every body's shapes.
template <typename Real, int ND, int NW, int NB>
__device__ __forceinline__ bool deposit_adjoint_w(const Real* J, int64_t jplane,
                                                  const Where3& wh, const Real* const x0[NB],
                                                  const Real* const x1[NB], const Real Q[NB],
                                                  const Real* const v[NB],
                                                  const PushConst<Real>& c, Real g0[NB][3],
                                                  Real g1[NB][3], Real gv[NB][3]) {
  const Real third = Real(1) / Real(3), sixth = Real(1) / Real(6);
  const int base = wh.base, sy = wh.sy;
  // component planes by pointer (their offsets may exceed 2^31), nodes by
  // 32-bit index
  const Real* const J1 = J + jplane;
  const Real* const J2 = J + 2 * jplane;
#pragma unroll
  for (int b = 0; b < NB; b++)
#pragma unroll
    for (int d = 0; d < 3; d++) g0[b][d] = g1[b][d] = gv[b][d] = Real(0);
  if constexpr (ND == 1) {
    Win<Real, NW> wx[NB];
#pragma unroll
    for (int b = 0; b < NB; b++)
      if (!win_build(x0[b][0], x1[b][0], wx[b]) || wx[b].lo != wx[0].lo) return false;
    const int o = base + wx[0].lo;
    // J_x(r) = fx C(r), r < NW - 1; J_y,z(r) = fv v_{y,z} (S0 + S1)(r) / 2
    Real L[NW];
    L[NW - 1] = Real(0);
    Real acc = 0;
#pragma unroll
    for (int r = NW - 2; r >= 0; r--) {
      acc += J[o + r];
      L[r] = acc;
    }
#pragma unroll
    for (int r = 0; r < NW; r++) {
      const Real ly = J1[o + r], lz = J2[o + r];
#pragma unroll
      for (int b = 0; b < NB; b++) {
        const Real fx = Q[b] * c.jf[0], fv = Q[b] * c.inv_dv;
        const Real A = Real(0.5) * (wx[b].S0[r] + wx[b].S1[r]);
        gv[b][1] += fv * ly * A;
        gv[b][2] += fv * lz * A;
        const Real t = Real(0.5) * fv * (v[b][1] * ly + v[b][2] * lz);
        const Real dS1 = fx * L[r] + t, dS0 = -fx * L[r] + t;
        g0[b][0] += dS0 * wx[b].D0[r];
        g1[b][0] += dS1 * wx[b].D1[r];
      }
    }
    return true;
  } else if constexpr (ND == 2) {
    Win<Real, NW> wx[NB], wy[NB];
#pragma unroll
    for (int b = 0; b < NB; b++)
      if (!win_build(x0[b][0], x1[b][0], wx[b]) || !win_build(x0[b][1], x1[b][1], wy[b]) ||
          wx[b].lo != wx[0].lo || wy[b].lo != wy[0].lo)
        return false;
    const int o = base + wx[0].lo + wy[0].lo * sy;
    Real fx[NB], fy[NB], fz[NB];
    Real G0x[NB][NW], G1x[NB][NW], G0y[NB][NW], G1y[NB][NW];
    Real Ax[NB][NW], Ay[NB][NW], DSx[NB][NW], DSy[NB][NW];
#pragma unroll
    for (int b = 0; b < NB; b++) {
      fx[b] = Q[b] * c.jf[0];
      fy[b] = Q[b] * c.jf[1];
      fz[b] = Q[b] * v[b][2] * c.inv_dv;
#pragma unroll
      for (int r = 0; r < NW; r++) {
        G0x[b][r] = G1x[b][r] = G0y[b][r] = G1y[b][r] = Real(0);
        Ax[b][r] = Real(0.5) * (wx[b].S0[r] + wx[b].S1[r]);
        Ay[b][r] = Real(0.5) * (wy[b].S0[r] + wy[b].S1[r]);
        DSx[b][r] = wx[b].S1[r] - wx[b].S0[r];
        DSy[b][r] = wy[b].S1[r] - wy[b].S0[r];
      }
    }
    // J_x(r, s) = fx Cx(r) Ay(s), r < NW - 1: Lx(r, s) suffix sums along x
#pragma unroll
    for (int s = 0; s < NW; s++) {
      Real acc = 0, Lx[NW];
      Lx[NW - 1] = Real(0);
#pragma unroll
      for (int r = NW - 2; r >= 0; r--) {
        acc += J[o + r + s * sy];
        Lx[r] = acc;
      }
#pragma unroll
      for (int b = 0; b < NB; b++) {
        Real sumDL = 0;
#pragma unroll
        for (int r = 0; r < NW; r++) {
          const Real t = fx[b] * Ay[b][s] * Lx[r];
          G1x[b][r] += t;
          G0x[b][r] -= t;
          sumDL += DSx[b][r] * Lx[r];
        }
        G0y[b][s] += Real(0.5) * fx[b] * sumDL;
        G1y[b][s] += Real(0.5) * fx[b] * sumDL;
      }
    }
    // J_y(r, s) = fy Cy(s) Ax(r), s < NW - 1: Ly(r, s) suffix sums along y
#pragma unroll
    for (int r = 0; r < NW; r++) {
      Real acc = 0, Ly[NW];
      Ly[NW - 1] = Real(0);
#pragma unroll
      for (int s = NW - 2; s >= 0; s--) {
        acc += J1[o + r + s * sy];
        Ly[s] = acc;
      }
#pragma unroll
      for (int b = 0; b < NB; b++) {
        Real sumDL = 0;
#pragma unroll
        for (int s = 0; s < NW; s++) {
          const Real t = fy[b] * Ax[b][r] * Ly[s];
          G1y[b][s] += t;
          G0y[b][s] -= t;
          sumDL += DSy[b][s] * Ly[s];
        }
        G0x[b][r] += Real(0.5) * fy[b] * sumDL;
        G1x[b][r] += Real(0.5) * fy[b] * sumDL;
      }
    }
    // J_z(r, s) = fz W(r, s), W = S0x S0y/3 + S0x S1y/6 + S1x S0y/6 + S1x S1y/3
#pragma unroll
    for (int s = 0; s < NW; s++)
#pragma unroll
      for (int r = 0; r < NW; r++) {
        const Real lz = J2[o + r + s * sy];
        if (lz == Real(0)) continue;
#pragma unroll
        for (int b = 0; b < NB; b++) {
          const Win<Real, NW>& X = wx[b];
          const Win<Real, NW>& Y = wy[b];
          const Real W = third * X.S0[r] * Y.S0[s] + sixth * X.S0[r] * Y.S1[s] +
                         sixth * X.S1[r] * Y.S0[s] + third * X.S1[r] * Y.S1[s];
          gv[b][2] += Q[b] * c.inv_dv * lz * W;
          const Real t = fz[b] * lz;
          G0x[b][r] += t * (third * Y.S0[s] + sixth * Y.S1[s]);
          G1x[b][r] += t * (sixth * Y.S0[s] + third * Y.S1[s]);
          G0y[b][s] += t * (third * X.S0[r] + sixth * X.S1[r]);
          G1y[b][s] += t * (sixth * X.S0[r] + third * X.S1[r]);
        }
      }
#pragma unroll
    for (int b = 0; b < NB; b++)
#pragma unroll
      for (int r = 0; r < NW; r++) {
        g0[b][0] += G0x[b][r] * wx[b].D0[r];
        g1[b][0] += G1x[b][r] * wx[b].D1[r];
        g0[b][1] += G0y[b][r] * wy[b].D0[r];
        g1[b][1] += G1y[b][r] * wy[b].D1[r];
      }
    return true;
  } else {
    Win<Real, NW> w[NB][3];
#pragma unroll
    for (int b = 0; b < NB; b++)
#pragma unroll
      for (int d = 0; d < 3; d++)
        if (!win_build(x0[b][d], x1[b][d], w[b][d]) || w[b][d].lo != w[0][d].lo) return false;
    const int st[3] = {1, sy, wh.sz};
    const int o = base + w[0][0].lo + w[0][1].lo * sy + w[0][2].lo * wh.sz;
    Real G0[NB][3][NW], G1[NB][3][NW];
#pragma unroll
    for (int b = 0; b < NB; b++)
#pragma unroll
      for (int d = 0; d < 3; d++)
#pragma unroll
        for (int r = 0; r < NW; r++) G0[b][d][r] = G1[b][d][r] = Real(0);
    // J_a(i_a, i_b, i_c) = Q jf_a C_a(i_a) M(i_b, i_c), C_a the running sum of
    // the shape change along a, (e1, e2) the transverse axes
#pragma unroll
    for (int a = 0; a < 3; a++) {
      const int e1 = a == 0 ? 1 : 0, e2 = a == 2 ? 1 : 2;
      const Real* Ja = J + a * jplane;
#pragma unroll
      for (int s = 0; s < NW; s++)
#pragma unroll
        for (int t = 0; t < NW; t++) {
          const int ob = o + s * st[e1] + t * st[e2];
          Real L[NW], acc = 0;
          L[NW - 1] = Real(0);
#pragma unroll
          for (int r = NW - 2; r >= 0; r--) {
            acc += Ja[ob + r * st[a]];
            L[r] = acc;
          }
#pragma unroll
          for (int b = 0; b < NB; b++) {
            const Win<Real, NW>& A = w[b][a];
            const Win<Real, NW>& B = w[b][e1];
            const Win<Real, NW>& E = w[b][e2];
            const Real f = Q[b] * c.jf[a];
            const Real M = third * B.S0[s] * E.S0[t] + sixth * B.S0[s] * E.S1[t] +
                           sixth * B.S1[s] * E.S0[t] + third * B.S1[s] * E.S1[t];
            Real P = 0;
#pragma unroll
            for (int r = 0; r < NW; r++) {
              const Real q = f * M * L[r];
              G1[b][a][r] += q;
              G0[b][a][r] -= q;
              P += (A.S1[r] - A.S0[r]) * L[r];
            }
            P *= f;
            G0[b][e1][s] += P * (third * E.S0[t] + sixth * E.S1[t]);
            G1[b][e1][s] += P * (sixth * E.S0[t] + third * E.S1[t]);
            G0[b][e2][t] += P * (third * B.S0[s] + sixth * B.S1[s]);
            G1[b][e2][t] += P * (sixth * B.S0[s] + third * B.S1[s]);
          }
        }
    }
#pragma unroll
    for (int b = 0; b < NB; b++)
#pragma unroll
      for (int d = 0; d < 3; d++)
#pragma unroll
        for (int r = 0; r < NW; r++) {
          g0[b][d] += G0[b][d][r] * w[b][d].D0[r];
          g1[b][d] += G1[b][d][r] * w[b][d].D1[r];
        }
    return true;
  }
}

// The deposit adjoint of one body on the three-node windows when it keeps
// its nearest node along every resolved axis (most bodies), else on four.
template <typename Real, int ND>
__device__ __forceinline__ bool deposit_adjoint(const Real* J, int64_t jplane, const Where3& wh,
                                                const Real x0[3], const Real x1[3], Real Q,
                                                const Real v[3], const PushConst<Real>& c,
                                                Real g0[3], Real g1[3], Real gv[3]) {
  bool keep = true;
#pragma unroll
  for (int d = 0; d < ND; d++) keep = keep && floor(x0[d] + Real(0.5)) == floor(x1[d] + Real(0.5));
  const Real* const a0[1] = {x0};
  const Real* const a1[1] = {x1};
  const Real* const av[1] = {v};
  const Real q[1] = {Q};
  Real h0[1][3], h1[1][3], hv[1][3];
  const bool ok = keep ? deposit_adjoint_w<Real, ND, 3, 1>(J, jplane, wh, a0, a1, q, av, c, h0, h1, hv)
                       : deposit_adjoint_w<Real, ND, 4, 1>(J, jplane, wh, a0, a1, q, av, c, h0, h1, hv);
#pragma unroll
  for (int d = 0; d < 3; d++) {
    g0[d] = h0[0][d];
    g1[d] = h1[0][d];
    gv[d] = hv[0][d];
  }
  return ok;
}

// Wall reflection as in the forward cycle; returns true if it reflected.
template <typename Real>
__device__ __forceinline__ bool reflect_wall(int periodic, int ci, int n, int pad, Real& off) {
  if (periodic) return false;
  const int wl = pad, wr = n - pad;
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

template <typename Real>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); w++) t += sh[w];
  __syncthreads();
  return t;
}

// What the reverse cycle of one particle reads from memory: its stored
// state at the start of the step and the adjoint of its state at the end.
// Loaded one particle ahead in the tiled kernel so that the loads overlap
// the previous particle's arithmetic.
template <typename Real>
struct PIn {
  uint32_t cell;
  Real off[3], u1[3], u2[3], dl[3], wc, w;
  Real loff[3], ldl[3], lu1[3], lu2[3];
};

template <typename Real, int ND, bool TWO>
__device__ __forceinline__ void load_in(const AdjState<Real>& st, const AdjState<Real>& lp,
                                        const PushConst<Real>& c, int64_t p, PIn<Real>& in) {
  in.cell = st.cell[p];
#pragma unroll
  for (int d = 0; d < 3; d++) {
    in.off[d] = d < ND ? st.off[d][p] : Real(0);
    in.loff[d] = d < ND ? lp.off[d][p] : Real(0);
  }
#pragma unroll
  for (int q = 0; q < 3; q++) {
    in.u1[q] = st.u1[q][p];
    in.lu1[q] = lp.u1[q][p];
    in.u2[q] = TWO ? st.u2[q][p] : Real(0);
    in.dl[q] = TWO ? st.dl[q][p] : Real(0);
    in.lu2[q] = TWO ? lp.u2[q][p] : Real(0);
    in.ldl[q] = TWO ? lp.dl[q][p] : Real(0);
  }
  in.wc = TWO ? (st.wc ? st.wc[p] : c.omega_c) : Real(0);
  in.w = st.w ? st.w[p] : Real(1);
}

// Tile of the workgroup in the tiled adjoint kernel: cells [x0, x0 + tx) x
// [y0, y0 + ty) and LDS copies of its nodes [x0 - 2, x0 + tx + 3) x
// [y0 - 2, y0 + ty + 3) (the reach of the gather and of the deposit window
// of a particle in the tile), `plane` values per component, row pitch
// `pitch`: the FP64 accumulator of the gather's transpose (6 planes), the
// fields E, B (6 planes) and the adjoint current (3 planes).
template <typename Real>
struct TileBox {
  double* lds;
  Real* f;   // staged E, B (1D and 2D)
  Real* lj;  // staged adjoint current (1D and 2D)
  int x0, y0, z0, tx, ty, tz, pitch, slab, plane;
};


// Adjoint of the per-body walls of a two-body ion along axis d (see the
// reverse sweep of adjoint_one).
template <typename Real>
__device__ __noinline__ void walls_adjoint(const PushConst<Real>& c, int d, bool w1, bool w2,
                                           Real& l_offn, Real& l_dln, Real& l_n1, Real& l_n2) {
  const Real lR = l_offn, ls = l_dln * c.dxs[d];
  Real lY1 = c.f2 * lR + ls, lY2 = c.f1 * lR - ls;
  if (w1) {
    lY1 = -lY1;
    l_n1 = -l_n1;
  }
  if (w2) {
    lY2 = -lY2;
    l_n2 = -l_n2;
  }
  l_offn = lY1 + lY2;
  l_dln = (c.f1 * lY1 - c.f2 * lY2) * c.idx[d];
}

// Reverse the cycle of particle p (see the file comment).
// IN_TILE: the particle's cell is in the workgroup's tile, so its fields,
// adjoint current and scatter live in the tile's LDS copies (known LDS
// addresses); otherwise everything goes through the global planes.
template <typename Real, int ND, bool TWO, bool IN_TILE>
__device__ __forceinline__ void adjoint_one(const GridInfo& g, const Planes<Real>& fg,
                                            const AdjState<Real>& st, const PushConst<Real>& c,
                                            const AdjState<Real>& lp, const Planes<Real>& l,
                                            int64_t p, const PIn<Real>& in,
                                            const TileBox<Real>& box, double& d_wc,
                                            double& d_nu, double& n_far) {
  do {
    // ---- stored state at the start of the step
    int ci[3] = {0, 0, 0};
    const uint32_t pk = in.cell;
    ci[0] = pk & ((1u << g.bits[0]) - 1u);
    if (ND > 1) ci[1] = (pk >> g.bits[0]) & ((1u << g.bits[1]) - 1u);
    if (ND > 2) ci[2] = pk >> (g.bits[0] + g.bits[1]);
    Real off[3] = {0, 0, 0}, u1[3], u2[3] = {0, 0, 0}, dl[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < ND; d++) off[d] = in.off[d];
#pragma unroll
    for (int q = 0; q < 3; q++) {
      u1[q] = in.u1[q];
      if (TWO) {
        u2[q] = in.u2[q];
        dl[q] = in.dl[q];
      }
    }
    const Real wc = in.wc;
    const Real W = in.w;
    bool ok = true, near = true;
    Real x1[3] = {0, 0, 0}, x2[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < ND; d++) {
      ok = ok && isfinite(off[d]) && off[d] >= Real(0) && off[d] <= Real(1);
      const Real sd = dl[d] * c.idx[d];
      if (TWO) near = near && fabs(sd) < Real(0.5);
      x1[d] = off[d] + (TWO ? c.f1 * sd : Real(0));
      x2[d] = off[d] - (TWO ? c.f2 * sd : Real(0));
    }
#pragma unroll
    for (int q = 0; q < 3; q++) ok = ok && isfinite(u1[q]) && isfinite(u2[q]) && isfinite(dl[q]);
    if (!ok) break;  // the forward cycle left it unchanged: identity
    if (TWO && !near) {
      // bodies half a cell or more apart: the forward took the far-body
      // path, which this reverse cycle does not cover; counted, and the
      // gradient run reports it
      n_far += 1.0;
      break;
    }
    // where the fields, the adjoint current and the scatter live: the
    // tile's LDS copies for a particle in the tile (in 3D only the scatter,
    // the fields and adjoint current being read from the global planes),
    // else the global planes
    Planes<Real> f = fg;
    const Real* LJ = l.J(0);
    int64_t jplane = l.plane;
    Sink<Real> k;
    k.l = l;
    k.gbase = (int)(g.origin + ci[0] + (ND > 1 ? (int64_t)ci[1] * g.sy : 0) +
                    (ND > 2 ? (int64_t)ci[2] * g.sz : 0));
    k.gsy = (int)g.sy;
    k.gsz = (int)g.sz;
    k.lds = nullptr;
    k.lbase = k.lsy = k.lsz = k.lplane = 0;
    Where3 wh{k.gbase, (int)g.sy, (int)g.sz};
    if constexpr (IN_TILE) {
      const int cx = ci[0] - box.x0, cy = ND > 1 ? ci[1] - box.y0 : 0;
      const int cz = ND > 2 ? ci[2] - box.z0 : 0;
      const int lidx = (cx + 2) + (ND > 1 ? (cy + 2) * box.pitch : 0) +
                       (ND > 2 ? (cz + 2) * box.slab : 0);
      k.lds = box.lds;
      k.lbase = lidx;
      k.lsy = box.pitch;
      k.lsz = box.slab;
      k.lplane = box.plane;
      if constexpr (ND < 3) {
        f = Planes<Real>{box.f, box.plane};
        LJ = box.lj;
        jplane = box.plane;
        wh = Where3{lidx, box.pitch, box.slab};
      }
    }

    // ---- forward recomputation
    Real G1[3], B1[3], G2[3] = {0, 0, 0}, B2[3] = {0, 0, 0};
    if (TWO)
      gather_values2<Real, ND>(f, wh, x1, x2, G1, B1, G2, B2);
    else
      gather_values<Real, ND>(f, wh, x1, G1, B1);
    Real E1[3], E2[3] = {0, 0, 0}, um1[3], um2[3] = {0, 0, 0};
    Real r2 = 0, rq = 1, soft = 1, kf = 0, iac2 = 0;
    if (TWO) {
      r2 = dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2];
      iac2 = ion_inv_ac2(c, st.wc != nullptr, wc);
      if (iac2 != Real(0)) {
        rq = rsq(Real(1) + r2 * iac2);
        soft = rq * rq * rq;
      }
      kf = -c.mr * wc * wc * soft;
    }
#pragma unroll
    for (int q = 0; q < 3; q++) {
      const Real F = kf * dl[q];
      E1[q] = G1[q] + (TWO ? F * c.inv_q1 : Real(0));
      um1[q] = u1[q] + c.a1 * E1[q];
      if (TWO) {
        E2[q] = G2[q] - F * c.inv_q2;
        um2[q] = u2[q] + c.a2 * E2[q];
      }
    }
    // friction on the relative momentum (identity when nu = 0)
    const Real nu = TWO ? c.nu + c.nu_per_omega * wc : Real(0);
    const Real Dn = (Real(1) - nu * c.half_dt) * rcp(Real(1) + nu * c.half_dt);
    Real vm1[3], vm2[3] = {0, 0, 0};
#pragma unroll
    for (int q = 0; q < 3; q++) {
      if (TWO) {
        const Real V = (c.m1 * um1[q] + c.m2 * um2[q]) * c.inv_mc;
        const Real w = (um1[q] - um2[q]) * Dn;
        vm1[q] = V + c.f1 * w;
        vm2[q] = V - c.f2 * w;
      } else {
        vm1[q] = um1[q];
      }
    }
    Real n1[3], n2[3] = {0, 0, 0}, v1[3], v2[3] = {0, 0, 0};
    boris_forward(vm1, c.a1, E1, B1, n1);
    if (TWO) boris_forward(vm2, c.a2, E2, B2, n2);
    {
      const Real i1 = rsq(Real(1) + n1[0] * n1[0] + n1[1] * n1[1] + n1[2] * n1[2]);
      const Real i2 = rsq(Real(1) + n2[0] * n2[0] + n2[1] * n2[1] + n2[2] * n2[2]);
#pragma unroll
      for (int q = 0; q < 3; q++) {
        v1[q] = n1[q] * i1;
        v2[q] = n2[q] * i2;
      }
    }
    Real dln[3], offn[3] = {0, 0, 0};
#pragma unroll
    for (int q = 0; q < 3; q++) dln[q] = TWO ? dl[q] + c.dt * (v1[q] - v2[q]) : Real(0);
    bool refl[3] = {false, false, false};
    unsigned walls = 0u;
#pragma unroll
    for (int d = 0; d < ND; d++) {
      const Real vc = TWO ? (c.m1 * v1[d] + c.m2 * v2[d]) * c.inv_mc : v1[d];
      offn[d] = off[d] + c.dt * vc * c.idx[d];
      if (!TWO) refl[d] = reflect_wall(g.periodic[d], ci[d], g.n[d], g.pad, offn[d]);
    }
    if (TWO) {
      // walls act on each body; the momenta flipped there are the stored
      // output, not the n1, n2 the reverse of v = u / gamma needs
      Real m1c[3] = {n1[0], n1[1], n1[2]}, m2c[3] = {n2[0], n2[1], n2[2]};
      walls = two_body_walls<Real, ND>(g, c, ci, offn, dln, m1c, m2c);
    }
    Real y1[3] = {0, 0, 0}, y2[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < ND; d++) {
      const Real sd = dln[d] * c.idx[d];
      y1[d] = offn[d] + (TWO ? c.f1 * sd : Real(0));
      y2[d] = offn[d] - (TWO ? c.f2 * sd : Real(0));
    }

    // ---- reverse
    Real l_off[3] = {0, 0, 0}, l_dl[3] = {0, 0, 0}, l_u1[3] = {0, 0, 0}, l_u2[3] = {0, 0, 0};
    Real l_offn[3] = {0, 0, 0}, l_dln[3] = {0, 0, 0}, l_n1[3], l_n2[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < ND; d++) l_offn[d] = in.loff[d];
#pragma unroll
    for (int q = 0; q < 3; q++) {
      l_n1[q] = in.lu1[q];
      if (TWO) {
        l_n2[q] = in.lu2[q];
        l_dln[q] = in.ldl[q];
      }
    }
    Real l_v1[3] = {0, 0, 0}, l_v2[3] = {0, 0, 0};
    if (c.deposit) {
      // one body at a time (loop not unrolled: one copy of the deposit
      // adjoint keeps the registers low); results to their body by selects
      const Real Q1 = st.w ? c.q1 * W : c.qw1, Q2 = st.w ? c.q2 * W : c.qw2;
#pragma unroll 1
      for (int body = 0; body < (TWO ? 2 : 1); body++) {
        Real xa[3], ya[3], va[3], g0[3], g1[3], gv[3];
#pragma unroll
        for (int q = 0; q < 3; q++) {
          xa[q] = body == 0 ? x1[q] : x2[q];
          ya[q] = body == 0 ? y1[q] : y2[q];
          va[q] = body == 0 ? v1[q] : v2[q];
        }
        if (deposit_adjoint<Real, ND>(LJ, jplane, wh, xa, ya, body == 0 ? Q1 : Q2, va, c, g0,
                                      g1, gv)) {
          const Real fs = body == 0 ? c.f1 : -c.f2;
#pragma unroll
          for (int d = 0; d < ND; d++) {
            l_offn[d] += g1[d];
            l_off[d] += g0[d];
            if (TWO) {
              l_dln[d] += fs * c.idx[d] * g1[d];
              l_dl[d] += fs * c.idx[d] * g0[d];
            }
          }
#pragma unroll
          for (int q = ND; q < 3; q++) {
            l_v1[q] += body == 0 ? gv[q] : Real(0);
            l_v2[q] += body == 0 ? Real(0) : gv[q];
          }
        }
      }
    }
    // walls.  A point particle: the reflected components change sign.  A
    // two-body ion: in body coordinates Y1 = R + f1 s, Y2 = R - f2 s
    // (s = delta / dx) a mirrored body's coordinate and momentum component
    // change sign; the adjoint goes to body coordinates (transpose of the
    // inverse map R = f2 Y1 + f1 Y2, s = Y1 - Y2), flips, and comes back.
#pragma unroll
    for (int d = 0; d < ND; d++) {
      if (!TWO && refl[d]) {
        l_offn[d] = -l_offn[d];
        l_n1[d] = -l_n1[d];
      }
      const bool w1 = (walls >> d) & 1u, w2 = (walls >> (4 + d)) & 1u;
      if (TWO && (w1 || w2)) {
        // FP32 builds inline this (a call would keep a copy of the kernel's
        // constants in scratch memory for the whole kernel); the FP64 builds
        // call walls_adjoint, as the compiler's back end rejects the
        // inlined form there ("operand has incorrect register class")
        if constexpr (sizeof(Real) == 4) {
          const Real lR = l_offn[d], ls = l_dln[d] * c.dxs[d];
          const Real s1 = w1 ? Real(-1) : Real(1), s2 = w2 ? Real(-1) : Real(1);
          const Real lY1 = s1 * (c.f2 * lR + ls), lY2 = s2 * (c.f1 * lR - ls);
          l_n1[d] *= s1;
          l_n2[d] *= s2;
          l_offn[d] = lY1 + lY2;
          l_dln[d] = (c.f1 * lY1 - c.f2 * lY2) * c.idx[d];
        } else {
          walls_adjoint(c, d, w1, w2, l_offn[d], l_dln[d], l_n1[d], l_n2[d]);
        }
      }
    }
    // move
#pragma unroll
    for (int d = 0; d < ND; d++) {
      l_off[d] += l_offn[d];
      const Real k = c.dt * c.idx[d] * l_offn[d];
      if (TWO) {
        l_v1[d] += k * c.m1 * c.inv_mc;
        l_v2[d] += k * c.m2 * c.inv_mc;
      } else {
        l_v1[d] += k;
      }
    }
    if (TWO)
#pragma unroll
      for (int q = 0; q < 3; q++) {
        l_dl[q] += l_dln[q];
        l_v1[q] += c.dt * l_dln[q];
        l_v2[q] -= c.dt * l_dln[q];
      }
    velocity_adjoint(n1, l_v1, l_n1);
    if (TWO) velocity_adjoint(n2, l_v2, l_n2);
    // Boris
    Real l_vm1[3] = {0, 0, 0}, l_vm2[3] = {0, 0, 0};
    Real l_E1[3] = {0, 0, 0}, l_E2[3] = {0, 0, 0}, l_B1[3] = {0, 0, 0}, l_B2[3] = {0, 0, 0};
    boris_adjoint(vm1, c.a1, B1, l_n1, l_vm1, l_E1, l_B1);
    if (TWO) boris_adjoint(vm2, c.a2, B2, l_n2, l_vm2, l_E2, l_B2);
    // friction
    Real l_um1[3], l_um2[3] = {0, 0, 0};
    if (TWO) {
      const Real dD = Real(-2) * c.half_dt * rcp((Real(1) + nu * c.half_dt) *
                                                 (Real(1) + nu * c.half_dt));
#pragma unroll
      for (int q = 0; q < 3; q++) {
        const Real lV = l_vm1[q] + l_vm2[q];
        const Real lw = c.f1 * l_vm1[q] - c.f2 * l_vm2[q];
        l_um1[q] = c.m1 * c.inv_mc * lV + Dn * lw;
        l_um2[q] = c.m2 * c.inv_mc * lV - Dn * lw;
        d_nu += (double)(lw * (um1[q] - um2[q]) * dD);
      }
    } else {
#pragma unroll
      for (int q = 0; q < 3; q++) l_um1[q] = l_vm1[q];
    }
    // half kicks
#pragma unroll
    for (int q = 0; q < 3; q++) {
      l_u1[q] += l_um1[q];
      l_E1[q] += c.a1 * l_um1[q];
      if (TWO) {
        l_u2[q] += l_um2[q];
        l_E2[q] += c.a2 * l_um2[q];
      }
    }
    // bond force: E1 = E(x1) + F / q1, E2 = E(x2) - F / q2, F = kf delta
    if (TWO) {
      Real lkf = 0;
#pragma unroll
      for (int q = 0; q < 3; q++) {
        const Real lF = c.inv_q1 * l_E1[q] - c.inv_q2 * l_E2[q];
        l_dl[q] += kf * lF;
        lkf += lF * dl[q];
      }
      d_wc += (double)(lkf * Real(-2) * c.mr * wc * soft);
      if (iac2 != Real(0)) {
        // soft = (1 + r2 / a_c^2)^{-3/2}
        const Real lsoft = lkf * (-c.mr * wc * wc);
        const Real rq5 = rq * rq * rq * rq * rq;
        const Real dsoft = Real(-1.5) * iac2 * rq5;
#pragma unroll
        for (int q = 0; q < 3; q++) l_dl[q] += Real(2) * dl[q] * lsoft * dsoft;
        // a derived a_c moves with omega_c: 1/a_c^2 = ac_k omega_c^{4/3},
        // d(1/a_c^2)/d omega_c = (4/3) (1/a_c^2) / omega_c
        if (c.ac_k != Real(0))
          d_wc += (double)(lsoft * (Real(-1.5) * r2 * rq5) * (Real(4) / Real(3)) * iac2 / wc);
      }
    }
    // gather
    Real lx1[3] = {0, 0, 0}, lx2[3] = {0, 0, 0};
    const Stencil<Real> t1 = stencil_at<Real, ND>(x1);
    if (TWO) {
      const Stencil<Real> t2 = stencil_at<Real, ND>(x2);
      if (same_nodes<Real, ND>(t1, t2)) {
        gather_adjoint<Real, ND, true>(f, k, wh, t1, l_E1, l_B1, t2, l_E2, l_B2, lx1, lx2);
      } else {
        // one body at a time, results to their body by selects
#pragma unroll 1
        for (int body = 0; body < 2; body++) {
          Real xb[3], lE[3], lB[3], lx[3] = {0, 0, 0};
#pragma unroll
          for (int q = 0; q < 3; q++) {
            xb[q] = body == 0 ? x1[q] : x2[q];
            lE[q] = body == 0 ? l_E1[q] : l_E2[q];
            lB[q] = body == 0 ? l_B1[q] : l_B2[q];
          }
          const Stencil<Real> tb = stencil_at<Real, ND>(xb);
          gather_adjoint<Real, ND, false>(f, k, wh, tb, lE, lB, tb, lE, lB, lx, lx);
#pragma unroll
          for (int q = 0; q < 3; q++) {
            lx1[q] = body == 0 ? lx[q] : lx1[q];
            lx2[q] = body == 0 ? lx2[q] : lx[q];
          }
        }
      }
    } else {
      gather_adjoint<Real, ND, false>(f, k, wh, t1, l_E1, l_B1, t1, l_E1, l_B1, lx1, lx1);
    }
#pragma unroll
    for (int d = 0; d < ND; d++) {
      l_off[d] += lx1[d] + lx2[d];
      if (TWO) l_dl[d] += c.idx[d] * (c.f1 * lx1[d] - c.f2 * lx2[d]);
    }
    // adjoint state at the start of the step
#pragma unroll
    for (int d = 0; d < ND; d++) lp.off[d][p] = l_off[d];
#pragma unroll
    for (int q = 0; q < 3; q++) {
      lp.u1[q][p] = l_u1[q];
      if (TWO) {
        lp.u2[q][p] = l_u2[q];
        lp.dl[q][p] = l_dl[q];
      }
    }
  } while (false);
}

template <typename Real, int ND, bool TWO>
__global__ void __launch_bounds__(256)
    k_adjoint_push(GridInfo g, Planes<Real> f, AdjState<Real> st, PushConst<Real> c,
                   AdjState<Real> lp, Planes<Real> l, double* dparam, double* dfar) {
  __shared__ double sh[4];
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double d_wc = 0.0, d_nu = 0.0, n_far = 0.0;
  TileBox<Real> box{};
  if (p < st.n) {
    PIn<Real> in;
    load_in<Real, ND, TWO>(st, lp, c, p, in);
    adjoint_one<Real, ND, TWO, false>(g, f, st, c, lp, l, p, in, box, d_wc, d_nu, n_far);
  }
  const double s_wc = block_sum<Real>(d_wc, sh);
  const double s_nu = block_sum<Real>(d_nu, sh);
  const double s_far = block_sum<Real>(n_far, sh);
  if (threadIdx.x == 0) {
    if (s_wc != 0.0) atomicAdd(&dparam[0], s_wc);
    if (s_nu != 0.0) atomicAdd(&dparam[1], s_nu);
    if (s_far != 0.0) atomicAdd(dfar, s_far);
  }
}

// Workgroups per CU the tiled kernel is built for: two (at most 256
// registers per lane, two waves per SIMD) where the reverse cycle fits
// them (FP32 in 1D and 2D), else one (the 3D and FP64 cycles keep more
// values live, and spill at 256).  At one wave per SIMD the 3D FP32 kernel
// issues the next particle's loads before this one's arithmetic (the
// registers of a second input set fit there; the FP64 kernels would spill).
template <typename Real, int ND>
struct AdjOccupancy {
  static constexpr int kBlocks = sizeof(Real) == 4 && ND < 3 ? 2 : 1;
  static constexpr bool kPrefetch = sizeof(Real) == 4 && ND == 3;
};

// One workgroup per tile of the sorted particle order: the gather's
// transpose of the tile's particles accumulates in an FP64 LDS patch
// (LDS atomics, 64-bit ones issue an order of magnitude faster than FP32
// ones on gfx950), flushed to the global adjoint planes once; particles
// that have left the tile since the sort scatter to the global planes
// directly.
template <typename Real, int ND, bool TWO>
__global__ void __launch_bounds__(256, (AdjOccupancy<Real, ND>::kBlocks))
    k_adjoint_tiled(GridInfo g, Planes<Real> f, AdjState<Real> st, PushConst<Real> c,
                    AdjState<Real> lp, Planes<Real> l, double* dparam, double* dfar,
                    const uint32_t* tile_off, AdjTiles tt) {
  extern __shared__ double patch[];
  __shared__ double sh[4];
  const int t = blockIdx.x;
  const int64_t p0 = tile_off[t], p1 = tile_off[t + 1];
  if (p0 == p1) return;  // uniform over the workgroup
  TileBox<Real> box;
  box.tx = tt.T[0];
  box.ty = ND > 1 ? tt.T[1] : 1;
  box.tz = ND > 2 ? tt.T[2] : 1;
  box.x0 = (t % tt.nt[0]) * tt.T[0];
  box.y0 = ND > 1 ? ((t / tt.nt[0]) % tt.nt[1]) * tt.T[1] : 0;
  box.z0 = ND > 2 ? (t / (tt.nt[0] * tt.nt[1])) * tt.T[2] : 0;
  box.pitch = box.tx + 5;
  box.slab = box.pitch * (ND > 1 ? box.ty + 5 : 1);
  box.plane = box.slab * (ND > 2 ? box.tz + 5 : 1);
  box.lds = patch;
  box.f = reinterpret_cast<Real*>(patch + 6 * box.plane);
  box.lj = box.f + 6 * box.plane;
  // zero the accumulator; in 1D and 2D stage E, B and the adjoint current of
  // the tile's reach (nodes beyond the guard layers, reachable only past a
  // partial last tile, read as zero)
  for (int q = threadIdx.x; q < 6 * box.plane; q += blockDim.x) {
    patch[q] = 0.0;
    if constexpr (ND < 3) {
      const int comp = q / box.plane, r = q % box.plane;
      const int gx = box.x0 - 2 + r % box.pitch, gy = box.y0 - 2 + r / box.pitch;
      const bool in = gx < g.n[0] + kGuard && (ND == 1 || gy < g.n[1] + kGuard);
      const int64_t o = g.origin + gx + (ND > 1 ? (int64_t)gy * g.sy : 0);
      box.f[q] = in ? f.base[comp * f.plane + o] : Real(0);
      if (comp < 3) box.lj[q] = in ? l.J(comp)[o] : Real(0);
    }
  }
  __syncthreads();
  double d_wc = 0.0, d_nu = 0.0, n_far = 0.0;
  constexpr bool kPrefetch = AdjOccupancy<Real, ND>::kPrefetch;
  PIn<Real> in;
  int64_t p = p0 + threadIdx.x;
  if (p < p1) load_in<Real, ND, TWO>(st, lp, c, p, in);
  for (; p < p1; p += blockDim.x) {
    PIn<Real> nx = in;
    if (kPrefetch && p + blockDim.x < p1) load_in<Real, ND, TWO>(st, lp, c, p + blockDim.x, nx);
    const uint32_t pk = in.cell;
    const int cx = (int)(pk & ((1u << g.bits[0]) - 1u)) - box.x0;
    const int cy = ND > 1 ? (int)((pk >> g.bits[0]) & ((1u << g.bits[1]) - 1u)) - box.y0 : 0;
    const int cz = ND > 2 ? (int)(pk >> (g.bits[0] + g.bits[1])) - box.z0 : 0;
    if (cx >= 0 && cx < box.tx && cy >= 0 && cy < box.ty && cz >= 0 && cz < box.tz)
      adjoint_one<Real, ND, TWO, true>(g, f, st, c, lp, l, p, in, box, d_wc, d_nu, n_far);
    else
      adjoint_one<Real, ND, TWO, false>(g, f, st, c, lp, l, p, in, box, d_wc, d_nu, n_far);
    if (kPrefetch)
      in = nx;
    else if (p + blockDim.x < p1)
      load_in<Real, ND, TWO>(st, lp, c, p + blockDim.x, in);
  }
  __syncthreads();
  // flush: patch node (px, py, pz) is global node (x0 - 2 + px, ...)
  for (int q = threadIdx.x; q < 6 * box.plane; q += blockDim.x) {
    const double v = patch[q];
    if (v == 0.0) continue;
    const int comp = q / box.plane, r = q % box.plane;
    const int px = r % box.pitch, py = (r / box.pitch) % (box.slab / box.pitch);
    const int pz = r / box.slab;
    const int gx = box.x0 - 2 + px, gy = box.y0 - 2 + py, gz = box.z0 - 2 + pz;
    if (gx < -kGuard || gx >= g.n[0] + kGuard) continue;
    if (ND > 1 && (gy < -kGuard || gy >= g.n[1] + kGuard)) continue;
    if (ND > 2 && (gz < -kGuard || gz >= g.n[2] + kGuard)) continue;
    const int64_t o = g.origin + gx + (ND > 1 ? (int64_t)gy * g.sy : 0) +
                      (ND > 2 ? (int64_t)gz * g.sz : 0);
    Real* F = l.base + comp * l.plane;
    unsafeAtomicAdd(F + o, (Real)v);
  }
  const double s_wc = block_sum<Real>(d_wc, sh);
  const double s_nu = block_sum<Real>(d_nu, sh);
  const double s_far = block_sum<Real>(n_far, sh);
  if (threadIdx.x == 0) {
    if (s_wc != 0.0) atomicAdd(&dparam[0], s_wc);
    if (s_nu != 0.0) atomicAdd(&dparam[1], s_nu);
    if (s_far != 0.0) atomicAdd(dfar, s_far);
  }
}

}  // namespace

template <typename Real>
void launch_adjoint_push(const GridInfo& g, const Real* fields, const AdjState<Real>& st,
                         const PushConst<Real>& c, const AdjState<Real>& lp, Real* lam,
                         double* dparam, double* dfar, const uint32_t* tile_off,
                         const AdjTiles& tt, hipStream_t stream) {
  if (st.n <= 0) return;
  const Planes<Real> f{const_cast<Real*>(fields), g.plane};
  const Planes<Real> l{lam, g.plane};
  const bool two = c.two_body != 0;
  if (tile_off) {
    const size_t ntile = adjoint_tiles(g, tt);
    const size_t lds = adjoint_lds_bytes(g, tt, sizeof(Real));
    dim3 grid((unsigned)ntile);
#define PIC_ADJ_TILED(ND_, TWO_)                                                               \
    {                                                                                          \
      const void* fn = (const void*)k_adjoint_tiled<Real, ND_, TWO_>;                          \
      (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);     \
      hipLaunchKernelGGL((k_adjoint_tiled<Real, ND_, TWO_>), grid, 256, lds, stream, g, f, st,  \
                         c, lp, l, dparam, dfar, tile_off, tt);                                \
    }
    if (g.nd == 1 && two) PIC_ADJ_TILED(1, true)
    if (g.nd == 1 && !two) PIC_ADJ_TILED(1, false)
    if (g.nd == 2 && two) PIC_ADJ_TILED(2, true)
    if (g.nd == 2 && !two) PIC_ADJ_TILED(2, false)
    if (g.nd == 3 && two) PIC_ADJ_TILED(3, true)
    if (g.nd == 3 && !two) PIC_ADJ_TILED(3, false)
#undef PIC_ADJ_TILED
    return;
  }
  dim3 grid((unsigned)((st.n + 255) / 256));
#define PIC_ADJ_GLOBAL(ND_, TWO_)                                                              \
  hipLaunchKernelGGL((k_adjoint_push<Real, ND_, TWO_>), grid, 256, 0, stream, g, f, st, c, lp, l, \
                     dparam, dfar)
  if (g.nd == 1 && two) PIC_ADJ_GLOBAL(1, true);
  if (g.nd == 1 && !two) PIC_ADJ_GLOBAL(1, false);
  if (g.nd == 2 && two) PIC_ADJ_GLOBAL(2, true);
  if (g.nd == 2 && !two) PIC_ADJ_GLOBAL(2, false);
  if (g.nd == 3 && two) PIC_ADJ_GLOBAL(3, true);
  if (g.nd == 3 && !two) PIC_ADJ_GLOBAL(3, false);
#undef PIC_ADJ_GLOBAL
}

size_t adjoint_tiles(const GridInfo& g, const AdjTiles& tt) {
  size_t n = 1;
  for (int d = 0; d < g.nd; d++) n *= (size_t)tt.nt[d];
  return n;
}

size_t adjoint_lds_bytes(const GridInfo& g, const AdjTiles& tt, size_t rsize) {
  // patch nodes: the tile plus 2 nodes below and 3 above per resolved axis
  size_t nodes = 1;
  for (int d = 0; d < g.nd; d++) nodes *= (size_t)tt.T[d] + 5;
  // FP64 accumulator (6 planes); in 1D and 2D also E, B (6) and the adjoint
  // current (3) in the working precision
  return nodes * (6 * sizeof(double) + (g.nd < 3 ? 9 * rsize : 0));
}

template void launch_adjoint_push<float>(const GridInfo&, const float*, const AdjState<float>&,
                                         const PushConst<float>&, const AdjState<float>&, float*,
                                         double*, double*, const uint32_t*, const AdjTiles&,
                                         hipStream_t);
template void launch_adjoint_push<double>(const GridInfo&, const double*, const AdjState<double>&,
                                          const PushConst<double>&, const AdjState<double>&,
                                          double*, double*, double*, const uint32_t*,
                                          const AdjTiles&, hipStream_t);

}  // namespace pic
