// fields.hip -- Yee leapfrog field update, periodic guard exchange, first-
// order Mur open faces with laser injection through x-min, and probes.
//
// The field planes are streamed once per half step; these kernels are
// bound by HBM bandwidth (one thread per interior node, x fastest, so a
// wavefront reads and writes 64 consecutive values of each plane).
#include "pic_internal.h"

namespace pic {

namespace {

template <typename Real>
__global__ void k_zero(Real* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = Real(0);
}

// Storage coordinate helpers: a guard plane of dim d is addressed by its
// layer index along d (in interior units, may be negative) and by a flat
// position over the full storage extent of the two other dims.
__device__ __forceinline__ int64_t plane_index(const GridInfo& g, int d, int layer, int64_t q) {
  int64_t stride_d = d == 0 ? 1 : (d == 1 ? g.sy : g.sz);
  int a_dim = d == 0 ? 1 : 0;
  int b_dim = d == 2 ? 1 : 2;
  int64_t na = g.st[a_dim];
  int64_t a = q % na, b = q / na;
  int64_t sa = a_dim == 0 ? 1 : g.sy;
  int64_t sb = b_dim == 1 ? g.sy : g.sz;
  return (int64_t)(layer + g.g[d]) * stride_d + a * sa + b * sb;
}

// copy guards of dim d from the opposite side: layers -G..-1 <- n-G..n-1
// and n..n+G-1 <- 0..G-1, over the full extent of the other dims
template <typename Real>
__global__ void k_fill_periodic(GridInfo g, int d, Real* c0, Real* c1, Real* c2, int ncomp) {
  int a_dim = d == 0 ? 1 : 0, b_dim = d == 2 ? 1 : 2;
  int64_t nplane = (int64_t)g.st[a_dim] * g.st[b_dim];
  int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t total = nplane * 2 * kGuard;
  if (tid >= total) return;
  int64_t q = tid % nplane;
  int l = (int)(tid / nplane);  // 0 .. 2G-1
  int layer, src;
  if (l < kGuard) {
    layer = -kGuard + l;
    src = layer + g.n[d];
  } else {
    layer = g.n[d] + (l - kGuard);
    src = layer - g.n[d];
  }
  int64_t di = plane_index(g, d, layer, q), si = plane_index(g, d, src, q);
  Real* cs[3] = {c0, c1, c2};
  for (int c = 0; c < ncomp && c < 3; c++) cs[c][di] = cs[c][si];
}

// add guards of dim d onto the interior layers they alias and clear them
template <typename Real>
__global__ void k_fold_periodic(GridInfo g, int d, Real* c0, Real* c1, Real* c2, int ncomp) {
  int a_dim = d == 0 ? 1 : 0, b_dim = d == 2 ? 1 : 2;
  int64_t nplane = (int64_t)g.st[a_dim] * g.st[b_dim];
  int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t total = nplane * 2 * kGuard;
  if (tid >= total) return;
  int64_t q = tid % nplane;
  int l = (int)(tid / nplane);
  int layer, dst;
  if (l < kGuard) {
    layer = -kGuard + l;
    dst = layer + g.n[d];
  } else {
    layer = g.n[d] + (l - kGuard);
    dst = layer - g.n[d];
  }
  int64_t si = plane_index(g, d, layer, q), di = plane_index(g, d, dst, q);
  Real* cs[3] = {c0, c1, c2};
  for (int c = 0; c < ncomp && c < 3; c++) {
    cs[c][di] += cs[c][si];
    cs[c][si] = Real(0);
  }
}

__device__ __forceinline__ void interior_ijk(const GridInfo& g, int64_t t, int& i, int& j, int& k) {
  i = (int)(t % g.n[0]);
  int64_t r = t / g.n[0];
  j = (int)(r % g.n[1]);
  k = (int)(r / g.n[1]);
}

// B -= (dt/2) curl E on the interior
template <typename Real, int ND>
__global__ void __launch_bounds__(256) k_b_half(GridInfo g, FieldPtrs<Real> f, Real h, Real ix,
                                                Real iy, Real iz) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
  if (t >= ncell) return;
  int i, j, k;
  interior_ijk(g, t, i, j, k);
  int64_t o = g.origin + i + j * g.sy + k * g.sz;
  const Real *Ex = f.E[0], *Ey = f.E[1], *Ez = f.E[2];
  Real ex = Ex[o], ey = Ey[o], ez = Ez[o];
  Real cx = 0, cy = 0, cz = 0;
  cy -= (Ez[o + 1] - ez) * ix;
  cz += (Ey[o + 1] - ey) * ix;
  if (ND > 1) {
    cx += (Ez[o + g.sy] - ez) * iy;
    cz -= (Ex[o + g.sy] - ex) * iy;
  }
  if (ND > 2) {
    cx -= (Ey[o + g.sz] - ey) * iz;
    cy += (Ex[o + g.sz] - ex) * iz;
  }
  f.B[0][o] -= h * cx;
  f.B[1][o] -= h * cy;
  f.B[2][o] -= h * cz;
}

// E += dt (curl B - J) on the interior
template <typename Real, int ND>
__global__ void __launch_bounds__(256) k_e_full(GridInfo g, FieldPtrs<Real> f, Real dt, Real ix,
                                                Real iy, Real iz) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
  if (t >= ncell) return;
  int i, j, k;
  interior_ijk(g, t, i, j, k);
  int64_t o = g.origin + i + j * g.sy + k * g.sz;
  const Real *Bx = f.B[0], *By = f.B[1], *Bz = f.B[2];
  Real bx = Bx[o], by = By[o], bz = Bz[o];
  Real cx = 0, cy = 0, cz = 0;
  cy -= (bz - Bz[o - 1]) * ix;
  cz += (by - By[o - 1]) * ix;
  if (ND > 1) {
    cx += (bz - Bz[o - g.sy]) * iy;
    cz -= (bx - Bx[o - g.sy]) * iy;
  }
  if (ND > 2) {
    cx -= (by - By[o - g.sz]) * iz;
    cy += (bx - Bx[o - g.sz]) * iz;
  }
  f.E[0][o] += dt * (cx - f.J[0][o]);
  f.E[1][o] += dt * (cy - f.J[1][o]);
  f.E[2][o] += dt * (cz - f.J[2][o]);
}

// interior face plane of dim d: (a, b) run over the interior of the other dims
__device__ __forceinline__ void face_ab(const GridInfo& g, int d, int64_t t, int& a, int& b,
                                        int& na) {
  int a_dim = d == 0 ? 1 : 0;
  na = g.n[a_dim];
  a = (int)(t % na);
  b = (int)(t / na);
}
__device__ __forceinline__ int64_t face_node(const GridInfo& g, int d, int p, int a, int b) {
  int i, j, k;
  if (d == 0) {
    i = p; j = a; k = b;
  } else if (d == 1) {
    i = a; j = p; k = b;
  } else {
    i = a; j = b; k = p;
  }
  return g.origin + i + (int64_t)j * g.sy + (int64_t)k * g.sz;
}

// The four uniform cubic B-spline basis functions that are non-zero on one
// knot interval, at the local coordinate u in [0, 1): weights of the
// coefficients m-3 .. m of the interval [m h, (m+1) h).
__device__ __forceinline__ void spline_segment(double u, double w[4]) {
  const double v = 1.0 - u;
  w[0] = v * v * v / 6.0;
  w[1] = (3.0 * u * u * u - 6.0 * u * u + 4.0) / 6.0;
  w[2] = (-3.0 * u * u * u + 3.0 * u * u + 3.0 * u + 1.0) / 6.0;
  w[3] = u * u * u / 6.0;
}

// Envelope of the laser at t' = tau in [0, t_env]: sin^2(pi tau / t_env),
// or the cubic B-spline series of the n_env coefficients (knots h apart).
__device__ __forceinline__ double envelope(const LaserDev& L, double tau) {
  if (L.n_env <= 0) {
    double s = sin(3.14159265358979323846 * tau / L.t_env);
    return s * s;
  }
  const double x = tau / L.h_env;
  const int m = (int)floor(x);
  double w[4];
  spline_segment(x - (double)m, w);
  double e = 0.0;
#pragma unroll
  for (int r = 0; r < 4; r++) {
    const int k = m - 3 + r;
    if (k >= 0 && k < L.n_env) e += L.env[k] * w[r];
  }
  return e;
}

__device__ __forceinline__ double laser_time(const LaserDev& L, double tau) {
  if (tau < 0.0 || tau > L.t_env) return 0.0;
  return L.a0 * envelope(L, tau) * sin(L.omega * tau + L.phase);
}

// Incident B of the laser (wave along +x, or oblique) for component a at
// interior index (i, j, k) with the B stagger of that component, as
// amp * laser_time(tau): amp holds the polarisation sign and the transverse
// profile (0 for the component the laser does not drive), tau the retarded
// time.
__device__ __forceinline__ void incident_parts(const GridInfo& g, const LaserDev& L, int a, int i,
                                               int j, int k, double t, double& amp,
                                               double& tau) {
  amp = 0.0;
  tau = -1.0;
  if (!L.on) return;
  int want = L.pol == 2 ? 1 : 2;
  if (a != want) return;
  // B_a is half-staggered along the two axes other than a
  double sx = 0.5, sy = a == 1 ? 0.0 : 0.5, sz = a == 2 ? 0.0 : 0.5;
  double x = ((double)i + sx) * g.dx[0];
  if (L.oblique) {
    // plane wave travelling at an angle toward +y: B = n x E (c = 1), so the
    // in-plane E gives B_z = |E| and E_z gives B_y = -cos(angle) E_z
    double y = g.nd > 1 ? ((double)j + sy) * g.dx[1] - L.yc : 0.0;
    tau = t - L.t_delay - (x * L.cos_a + y * L.sin_a);
    amp = a == 2 ? 1.0 : -L.cos_a;
    return;
  }
  double prof = 1.0;
  if (L.waist > 0.0) {
    double r2 = 0.0;
    if (g.nd > 1) {
      double y = ((double)j + sy) * g.dx[1] - L.yc;
      r2 += y * y;
    }
    if (g.nd > 2) {
      double z = ((double)k + sz) * g.dx[2] - L.zc;
      r2 += z * z;
    }
    prof = exp(-r2 / (L.waist * L.waist));
  }
  tau = t - L.t_delay - x;
  amp = a == 2 ? prof : -prof;
}

__device__ __forceinline__ double b_incident(const GridInfo& g, const LaserDev& L, int a, int i,
                                             int j, int k, double t) {
  double amp, tau;
  incident_parts(g, L, a, i, j, k, t, amp, tau);
  return amp == 0.0 ? 0.0 : amp * laser_time(L, tau);
}

// Add coef * d(b_incident)/d(env[m]) to acc[m] for the (at most four)
// spline coefficients that the incident field at (i, j, k, t) depends on.
__device__ __forceinline__ void b_incident_grad(const GridInfo& g, const LaserDev& L, int a, int i,
                                                int j, int k, double t, double coef,
                                                double* acc) {
  double amp, tau;
  incident_parts(g, L, a, i, j, k, t, amp, tau);
  if (amp == 0.0 || L.n_env <= 0 || tau < 0.0 || tau > L.t_env) return;
  const double base = coef * amp * L.a0 * sin(L.omega * tau + L.phase);
  const double x = tau / L.h_env;
  const int m = (int)floor(x);
  double w[4];
  spline_segment(x - (double)m, w);
#pragma unroll
  for (int r = 0; r < 4; r++) {
    const int kk = m - 3 + r;
    if (kk >= 0 && kk < L.n_env) atomicAdd(&acc[kk], base * w[r]);
  }
}

// Mur condition on the scattered tangential B at the ghost half a cell
// below the low face of dim d (after the first B half step).
template <typename Real>
__global__ void k_mur_low_b(GridInfo g, FieldPtrs<Real> f, int d, Real* prev0, Real* prev1,
                            LaserDev L, int64_t step) {
  int a_dim = d == 0 ? 1 : 0, b_dim = d == 2 ? 1 : 2;
  int64_t np = (int64_t)g.n[a_dim] * g.n[b_dim];
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * np) return;
  int q = (int)(t / np);
  int64_t pi = t % np;
  int a, b, na;
  face_ab(g, d, pi, a, b, na);
  int comp = q == 0 ? (d == 0 ? 1 : 0) : (d == 2 ? 1 : 2);
  Real* Bf = f.B[comp];
  Real* prev = q == 0 ? prev0 : prev1;
  double dt = g.dt, dx = g.dx[d];
  double kc = (dt - dx) / (dt + dx);
  int64_t fg = face_node(g, d, -1, a, b), f1 = face_node(g, d, 0, a, b);
  double ig_m = 0, ig_p = 0, i1_m = 0, i1_p = 0;
  if (d == 0 && L.on) {
    double tn = (double)step * dt;
    int ig = -1, i1 = 0;
    int jj = d == 0 ? a : 0, kk = d == 0 ? b : 0;
    ig_m = b_incident(g, L, comp, ig, jj, kk, tn - 0.5 * dt);
    ig_p = b_incident(g, L, comp, ig, jj, kk, tn + 0.5 * dt);
    i1_m = b_incident(g, L, comp, i1, jj, kk, tn - 0.5 * dt);
    i1_p = b_incident(g, L, comp, i1, jj, kk, tn + 0.5 * dt);
  }
  double s1_old = (double)prev[pi] - i1_m;
  double sg_old = (double)Bf[fg] - ig_m;
  double s1_new = (double)Bf[f1] - i1_p;
  double sg_new = s1_old + kc * (s1_new - sg_old);
  Bf[fg] = (Real)(sg_new + ig_p);
  prev[pi] = Bf[f1];
}

template <typename Real>
__global__ void k_save_high_e(GridInfo g, FieldPtrs<Real> f, int d, Real* s0, Real* s1) {
  int a_dim = d == 0 ? 1 : 0, b_dim = d == 2 ? 1 : 2;
  int64_t np = (int64_t)g.n[a_dim] * g.n[b_dim];
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * np) return;
  int q = (int)(t / np);
  int64_t pi = t % np;
  int a, b, na;
  face_ab(g, d, pi, a, b, na);
  int comp = q == 0 ? (d == 0 ? 1 : 0) : (d == 2 ? 1 : 2);
  Real* save = q == 0 ? s0 : s1;
  save[pi] = f.E[comp][face_node(g, d, g.n[d] - 1, a, b)];
}

// Mur condition on the tangential E at the ghost on the high face of dim d
template <typename Real>
__global__ void k_mur_high_e(GridInfo g, FieldPtrs<Real> f, int d, const Real* s0,
                             const Real* s1) {
  int a_dim = d == 0 ? 1 : 0, b_dim = d == 2 ? 1 : 2;
  int64_t np = (int64_t)g.n[a_dim] * g.n[b_dim];
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * np) return;
  int q = (int)(t / np);
  int64_t pi = t % np;
  int a, b, na;
  face_ab(g, d, pi, a, b, na);
  int comp = q == 0 ? (d == 0 ? 1 : 0) : (d == 2 ? 1 : 2);
  const Real* save = q == 0 ? s0 : s1;
  double kc = (g.dt - g.dx[d]) / (g.dt + g.dx[d]);
  Real* Ef = f.E[comp];
  int64_t fg = face_node(g, d, g.n[d], a, b), f1 = face_node(g, d, g.n[d] - 1, a, b);
  Ef[fg] = (Real)((double)save[pi] + kc * ((double)Ef[f1] - (double)Ef[fg]));
}

// ---------------------------------------------------------------------------
// One field step in one pass over a tile of cells: B half step, E full step
// with J, B half step, with the Mur faces (and the laser of x-min) that sit
// between them.  The first-half B and the new E stay in LDS; E and B are read
// from one buffer and written to the other (neighbouring tiles read this
// tile's old values in their halos while it runs), the Mur history of the
// low faces likewise.  Per cell it reads E, B, J and writes E, B once.
template <typename Real, int ND>
struct YeeTile {
  static constexpr int TX = ND == 1 ? 512 : 64;
  static constexpr int TY = ND == 1 ? 1 : 8;
  // LDS regions per component, along each resolved dim: old E on
  // [-1, T + 1], first-half B on [-1, T], new E on [0, T]
  static constexpr int EX = TX + 3, EY = ND > 1 ? TY + 3 : 1;
  static constexpr int BX = TX + 2, BY = ND > 1 ? TY + 2 : 1;
  static constexpr int PX = TX + 1, PY = ND > 1 ? TY + 1 : 1;
  static constexpr int NE = EX * EY, NB = BX * BY, NP = PX * PY;
  static constexpr size_t lds = (size_t)3 * (NE + NB + NP) * sizeof(Real);
};

template <typename Real>
struct MurHistory {
  Real* in[3][2];   // B just inside each low open face after the last step's first half
  Real* out[3][2];  // the same after this step's
};

// curl E at a B node (forward differences) and curl B at an E node
// (backward differences), from planes with strides 1 (x) and sy (y)
template <typename Real, int ND>
__device__ __forceinline__ void curl_fwd(const Real* Ex, const Real* Ey, const Real* Ez, int e,
                                         int sy, Real ix, Real iy, Real& cx, Real& cy,
                                         Real& cz) {
  const Real ex = Ex[e], ey = Ey[e], ez = Ez[e];
  cx = 0;
  cy = 0;
  cz = 0;
  cy -= (Ez[e + 1] - ez) * ix;
  cz += (Ey[e + 1] - ey) * ix;
  if (ND > 1) {
    cx += (Ez[e + sy] - ez) * iy;
    cz -= (Ex[e + sy] - ex) * iy;
  }
}

template <typename Real, int ND>
__device__ __forceinline__ void curl_bwd(const Real* Bx, const Real* By, const Real* Bz, int b,
                                         int sy, Real ix, Real iy, Real& cx, Real& cy,
                                         Real& cz) {
  const Real bx = Bx[b], by = By[b], bz = Bz[b];
  cx = 0;
  cy = 0;
  cz = 0;
  cy -= (bz - Bz[b - 1]) * ix;
  cz += (by - By[b - 1]) * ix;
  if (ND > 1) {
    cx += (bz - Bz[b - sy]) * iy;
    cz -= (bx - Bx[b - sy]) * iy;
  }
}

// 1D and 2D (the 3D field step keeps its three streaming passes, which
// stay at the bandwidth the three-dimensional halos of one pass would
// spend); x is dim 0, y dim 1, and the tangential components of the x and
// y faces are (1, 2) and (0, 2).
template <typename Real, int ND>
__global__ void __launch_bounds__(256) k_yee_fused(GridInfo g, FieldPtrs<Real> fi,
                                                   FieldPtrs<Real> fo, MurHistory<Real> mh,
                                                   LaserDev L, int64_t step, Real h, Real dt,
                                                   Real ix, Real iy) {
  static_assert(ND == 1 || ND == 2, "one-pass field step in 1D and 2D");
  using T = YeeTile<Real, ND>;
  extern __shared__ __align__(16) unsigned char yee_lds[];
  Real* sE = reinterpret_cast<Real*>(yee_lds);  // [3][NE]
  Real* sB = sE + 3 * T::NE;                      // [3][NB]
  Real* sP = sB + 3 * T::NB;                      // [3][NP]
  const int ntx = (g.n[0] + T::TX - 1) / T::TX;
  const int nty = ND > 1 ? (g.n[1] + T::TY - 1) / T::TY : 1;
  // consecutive tiles on one XCD (workgroups go round-robin over the 8),
  // so that neighbours' halos meet in the same L2
  const int64_t ntiles = (int64_t)ntx * nty;
  const int64_t b = blockIdx.x, xcd = b & 7, per = ntiles >> 3, rem = ntiles & 7;
  const int64_t tile = xcd * per + (xcd < rem ? xcd : rem) + (b >> 3);
  const int ox = (int)(tile % ntx) * T::TX, oy = ND > 1 ? (int)(tile / ntx) * T::TY : 0;
  const int ex = min(T::TX, g.n[0] - ox), ey = ND > 1 ? min(T::TY, g.n[1] - oy) : 1;
  const bool px = g.periodic[0], py = ND > 1 && g.periodic[1];
  auto sidx = [&](int x, int y) -> int64_t {
    return g.origin + (ox + x) + (int64_t)(oy + y) * g.sy;
  };
  auto eix = [](int x, int y) { return (x + 1) + (ND > 1 ? (y + 1) * T::EX : 0); };
  auto bix = [](int x, int y) { return (x + 1) + (ND > 1 ? (y + 1) * T::BX : 0); };
  auto pix = [](int x, int y) { return x + (ND > 1 ? y * T::PX : 0); };

  // Every global load of the tile is issued before the first barrier: old
  // E into LDS, and into registers the old B of the positions this thread
  // advances in 2 and the J of those it advances in 3.
  constexpr int KE = (T::NE + 255) / 256, KB = (T::NB + 255) / 256, KP = (T::NP + 255) / 256;
  Real rb[KB][3], rj[KP][3];
  bool vb[KB], vp[KP];
  // 2's positions: B after the first half step on [-1, ext] (the low guard
  // of an open face takes its Mur value from the face node, in 2)
#pragma unroll
  for (int k = 0; k < KB; k++) {
    const int q = threadIdx.x + 256 * k;
    const int x = q % T::BX - 1, y = ND > 1 ? q / T::BX - 1 : 0;
    const bool v = q < T::NB && x <= ex && (ND < 2 || y <= ey) && (px || ox + x >= 0) &&
                   (ND < 2 || py || oy + y >= 0);
    vb[k] = v;
    const int64_t si = v ? sidx(x, y) : g.origin;
#pragma unroll
    for (int c = 0; c < 3; c++) rb[k][c] = fi.B[c][si];
  }
  // 3's positions: new E on [0, ext] (the high guard of an open face takes
  // its Mur value from the node below, in 3); J at a periodic guard is read
  // at its interior image (the folded guards are zero)
#pragma unroll
  for (int k = 0; k < KP; k++) {
    const int q = threadIdx.x + 256 * k;
    const int x = q % T::PX, y = ND > 1 ? q / T::PX : 0;
    int gx = ox + x, gy = oy + y;
    bool v = q < T::NP && x <= ex && (ND < 2 || y <= ey);
    if (gx >= g.n[0]) {
      if (px)
        gx -= g.n[0];
      else
        v = false;
    }
    if (ND > 1 && gy >= g.n[1]) {
      if (py)
        gy -= g.n[1];
      else
        v = false;
    }
    vp[k] = v;
    const int64_t sj = v ? g.origin + gx + (int64_t)gy * g.sy : g.origin;
#pragma unroll
    for (int c = 0; c < 3; c++) rj[k][c] = fi.J[c][sj];
  }
  // 1. old E on [-1, ext + 1] (guard layers hold the periodic images)
#pragma unroll
  for (int k = 0; k < KE; k++) {
    const int q = threadIdx.x + 256 * k;
    const int x = q % T::EX - 1, y = ND > 1 ? q / T::EX - 1 : 0;
    if (q >= T::NE || x > ex + 1 || (ND > 1 && y > ey + 1)) continue;
    const int64_t si = sidx(x, y);
#pragma unroll
    for (int c = 0; c < 3; c++) sE[c * T::NE + q] = fi.E[c][si];
  }
  __syncthreads();

  // 2. B after the first half step
#pragma unroll
  for (int k = 0; k < KB; k++) {
    if (!vb[k]) continue;
    const int q = threadIdx.x + 256 * k;
    const int x = q % T::BX - 1, y = ND > 1 ? q / T::BX - 1 : 0;
    Real cx, cy, cz;
    curl_fwd<Real, ND>(sE, sE + T::NE, sE + 2 * T::NE, eix(x, y), T::EX, ix, iy, cx, cy, cz);
    sB[q] = rb[k][0] - h * cx;
    sB[T::NB + q] = rb[k][1] - h * cy;
    sB[2 * T::NB + q] = rb[k][2] - h * cz;
  }
  __syncthreads();

  // 2b. Mur on the tangential B half a cell below each open low face this
  //     tile touches (with the incident laser B at x-min)
  for (int d = 0; d < ND; d++) {
    if ((d == 0 ? px : py) || (d == 0 ? ox : oy) != 0) continue;
    // face nodes along the other dim over the B region [-1, ext]
    const int nf = ND > 1 ? (d == 0 ? ey : ex) + 2 : 1;
    const int na = d == 0 ? g.n[1] : g.n[0];
    const bool pa = d == 0 ? py : px;
    const int oa = d == 0 ? oy : ox, ea = d == 0 ? ey : ex;
    const double dtd = g.dt, dxd = g.dx[d], kc = (dtd - dxd) / (dtd + dxd);
    for (int q = threadIdx.x; q < 2 * nf; q += 256) {
      const int qq = q / nf, la = ND > 1 ? q % nf - 1 : 0;
      // the face node's coordinate along the face, in the interior range
      // (a periodic image maps to it); the corners of two open faces are unused
      int ga = oa + la;
      if (ND > 1 && (ga < 0 || ga >= na)) {
        if (!pa) continue;
        ga = ga < 0 ? ga + na : ga - na;
      }
      const int comp = qq == 0 ? (d == 0 ? 1 : 0) : 2;
      const int b1 = d == 0 ? bix(0, la) : bix(la, 0);
      const int bg = d == 0 ? b1 - 1 : b1 - T::BX;
      const int64_t sg = d == 0 ? g.origin - 1 + (int64_t)ga * g.sy : g.origin + ga - g.sy;
      double ig_m = 0, ig_p = 0, i1_m = 0, i1_p = 0;
      if (d == 0 && L.on) {
        const double tn = (double)step * dtd;
        ig_m = b_incident(g, L, comp, -1, ga, 0, tn - 0.5 * dtd);
        ig_p = b_incident(g, L, comp, -1, ga, 0, tn + 0.5 * dtd);
        i1_m = b_incident(g, L, comp, 0, ga, 0, tn - 0.5 * dtd);
        i1_p = b_incident(g, L, comp, 0, ga, 0, tn + 0.5 * dtd);
      }
      const Real face = sB[comp * T::NB + b1];
      const double s1_old = (double)mh.in[d][qq][ga] - i1_m;
      const double sg_old = (double)fi.B[comp][sg] - ig_m;
      const double s1_new = (double)face - i1_p;
      const double sg_new = s1_old + kc * (s1_new - sg_old);
      const Real v = (Real)(sg_new + ig_p);
      sB[comp * T::NB + bg] = v;
      if (ND < 2 || (la >= 0 && la < ea)) {  // this tile's own face nodes
        fo.B[comp][sg] = v;
        mh.out[d][qq][ga] = face;
      }
    }
  }
  __syncthreads();

  // 3. new E
#pragma unroll
  for (int k = 0; k < KP; k++) {
    if (!vp[k]) continue;
    const int q = threadIdx.x + 256 * k;
    const int x = q % T::PX, y = ND > 1 ? q / T::PX : 0;
    Real cx, cy, cz;
    curl_bwd<Real, ND>(sB, sB + T::NB, sB + 2 * T::NB, bix(x, y), T::BX, ix, iy, cx, cy, cz);
    const int e = eix(x, y);
    sP[q] = sE[e] + dt * (cx - rj[k][0]);
    sP[T::NP + q] = sE[T::NE + e] + dt * (cy - rj[k][1]);
    sP[2 * T::NP + q] = sE[2 * T::NE + e] + dt * (cz - rj[k][2]);
  }
  __syncthreads();

  // 3b. Mur on the tangential E at the guard of each open high face
  for (int d = 0; d < ND; d++) {
    if ((d == 0 ? px : py) || (d == 0 ? ox + ex : oy + ey) != (d == 0 ? g.n[0] : g.n[1]))
      continue;
    const int nf = ND > 1 ? (d == 0 ? ey : ex) + 1 : 1;
    const int na = d == 0 ? g.n[1] : g.n[0];
    const bool pa = d == 0 ? py : px;
    const int oa = d == 0 ? oy : ox, ea = d == 0 ? ey : ex;
    const double kc = (g.dt - g.dx[d]) / (g.dt + g.dx[d]);
    for (int q = threadIdx.x; q < 2 * nf; q += 256) {
      const int qq = q / nf, la = ND > 1 ? q % nf : 0;
      if (ND > 1 && !pa && oa + la >= na) continue;  // corner of two open faces (unused)
      const int comp = qq == 0 ? (d == 0 ? 1 : 0) : 2;
      const int xg = d == 0 ? ex : la, yg = d == 0 ? la : ey;
      const int pg = pix(xg, yg), eg = eix(xg, yg);
      const int p1 = d == 0 ? pg - 1 : pg - T::PX, e1 = d == 0 ? eg - 1 : eg - T::EX;
      const Real v = (Real)((double)sE[comp * T::NE + e1] +
                            kc * ((double)sP[comp * T::NP + p1] - (double)sE[comp * T::NE + eg]));
      sP[comp * T::NP + pg] = v;
      if (ND < 2 || la < ea) fo.E[comp][sidx(xg, yg)] = v;
    }
  }
  __syncthreads();

  // 4. B after the second half step, and the new E, on the tile's cells
#pragma unroll
  for (int q = threadIdx.x; q < T::TX * T::TY; q += 256) {
    const int x = q % T::TX, y = ND > 1 ? q / T::TX : 0;
    if (x >= ex || (ND > 1 && y >= ey)) continue;
    const int p = pix(x, y), bb = bix(x, y);
    Real cx, cy, cz;
    curl_fwd<Real, ND>(sP, sP + T::NP, sP + 2 * T::NP, p, T::PX, ix, iy, cx, cy, cz);
    const int64_t si = sidx(x, y);
    fo.B[0][si] = sB[bb] - h * cx;
    fo.B[1][si] = sB[T::NB + bb] - h * cy;
    fo.B[2][si] = sB[2 * T::NB + bb] - h * cz;
    fo.E[0][si] = sP[p];
    fo.E[1][si] = sP[T::NP + p];
    fo.E[2][si] = sP[2 * T::NP + p];
  }
}

template <typename Real>
__global__ void k_probes(GridInfo g, FieldPtrs<Real> f, int nprobe, const int* comp,
                         const int64_t* index, Real* buf, int64_t max_steps, int64_t rec) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nprobe) return;
  int c = comp[p];
  const Real* F = c < 3 ? f.E[c] : f.B[c - 3];
  buf[(int64_t)p * max_steps + rec] = F[index[p]];
}

// ------------------------------------------------- adjoint (transposed) operators
//
// Each kernel below applies the transpose of one linear field operation of
// the step to the adjoint fields lE, lB (same layout as E, B).  They run
// over the nodes whose adjoint value changes and gather the contributions
// from the nodes that the forward operation wrote, so no atomics are
// needed.

// Node (i, j, k) of the range [lo, lo + n + 1) in each resolved dimension
// (one extra layer): returns false past the end.
__device__ __forceinline__ bool ext_ijk(const GridInfo& g, int64_t t, int lo, int& i, int& j,
                                        int& k) {
  const int ex = g.n[0] + 1, ey = g.nd > 1 ? g.n[1] + 1 : 1, ez = g.nd > 2 ? g.n[2] + 1 : 1;
  if (t >= (int64_t)ex * ey * ez) return false;
  i = (int)(t % ex) + lo;
  int64_t r = t / ex;
  j = g.nd > 1 ? (int)(r % ey) + lo : 0;
  k = g.nd > 2 ? (int)(r / ey) + lo : 0;
  return true;
}

__device__ __forceinline__ bool interior(const GridInfo& g, int i, int j, int k) {
  return i >= 0 && i < g.n[0] && j >= 0 && j < g.n[1] && k >= 0 && k < g.n[2];
}

// Transpose of B -= h curl E on the interior: lE += -h curl^T lB, over the
// E nodes that the curl reads (interior plus one layer above it).
template <typename Real, int ND>
__global__ void __launch_bounds__(256) k_b_half_adj(GridInfo g, FieldPtrs<Real> l, Real h,
                                                    Real ix, Real iy, Real iz) {
  int i, j, k;
  if (!ext_ijk(g, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, 0, i, j, k)) return;
  const int64_t o = g.origin + i + j * g.sy + k * g.sz;
  const bool in0 = interior(g, i, j, k);
  const bool inx = interior(g, i - 1, j, k);
  const bool iny = ND > 1 && interior(g, i, j - 1, k);
  const bool inz = ND > 2 && interior(g, i, j, k - 1);
  const Real *Bx = l.B[0], *By = l.B[1], *Bz = l.B[2];
  Real ax = 0, ay = 0, az = 0;
  // from B_y -= h [-(Ez[o+1] - Ez[o]) ix + (Ex[o+sz] - Ex[o]) iz]
  // and B_z -= h [(Ey[o+1] - Ey[o]) ix - (Ex[o+sy] - Ex[o]) iy]
  // and B_x -= h [(Ez[o+sy] - Ez[o]) iy - (Ey[o+sz] - Ey[o]) iz]
  if (in0) {
    az -= h * ix * By[o];
    ay += h * ix * Bz[o];
    if (ND > 1) {
      ax -= h * iy * Bz[o];
      az += h * iy * Bx[o];
    }
    if (ND > 2) {
      ax += h * iz * By[o];
      ay -= h * iz * Bx[o];
    }
  }
  if (inx) {
    az += h * ix * By[o - 1];
    ay -= h * ix * Bz[o - 1];
  }
  if (iny) {
    ax += h * iy * Bz[o - g.sy];
    az -= h * iy * Bx[o - g.sy];
  }
  if (inz) {
    ax -= h * iz * By[o - g.sz];
    ay += h * iz * Bx[o - g.sz];
  }
  l.E[0][o] += ax;
  l.E[1][o] += ay;
  l.E[2][o] += az;
}

// Transpose of E += dt (curl B - J) on the interior: lB += dt curl^T lE over
// the B nodes that the curl reads (interior plus one layer below it), and
// lJ = -dt lE on the interior.
template <typename Real, int ND>
__global__ void __launch_bounds__(256) k_e_full_adj(GridInfo g, FieldPtrs<Real> l, Real dt,
                                                    Real ix, Real iy, Real iz) {
  int i, j, k;
  if (!ext_ijk(g, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, -1, i, j, k)) return;
  const int64_t o = g.origin + i + j * g.sy + k * g.sz;
  const bool in0 = interior(g, i, j, k);
  const bool inx = interior(g, i + 1, j, k);
  const bool iny = ND > 1 && interior(g, i, j + 1, k);
  const bool inz = ND > 2 && interior(g, i, j, k + 1);
  const Real *Ex = l.E[0], *Ey = l.E[1], *Ez = l.E[2];
  Real bx = 0, by = 0, bz = 0;
  // E_x += dt [(Bz[o] - Bz[o-sy]) iy - (By[o] - By[o-sz]) iz]
  // E_y += dt [-(Bz[o] - Bz[o-1]) ix + (Bx[o] - Bx[o-sz]) iz]
  // E_z += dt [(By[o] - By[o-1]) ix - (Bx[o] - Bx[o-sy]) iy]
  if (in0) {
    bz -= dt * ix * Ey[o];
    by += dt * ix * Ez[o];
    if (ND > 1) {
      bz += dt * iy * Ex[o];
      bx -= dt * iy * Ez[o];
    }
    if (ND > 2) {
      by -= dt * iz * Ex[o];
      bx += dt * iz * Ey[o];
    }
    l.J[0][o] = -dt * Ex[o];
    l.J[1][o] = -dt * Ey[o];
    l.J[2][o] = -dt * Ez[o];
  }
  if (inx) {
    bz += dt * ix * Ey[o + 1];
    by -= dt * ix * Ez[o + 1];
  }
  if (iny) {
    bz -= dt * iy * Ex[o + g.sy];
    bx += dt * iy * Ez[o + g.sy];
  }
  if (inz) {
    by += dt * iz * Ex[o + g.sz];
    bx -= dt * iz * Ey[o + g.sz];
  }
  l.B[0][o] += bx;
  l.B[1][o] += by;
  l.B[2][o] += bz;
}

// Transpose of the Mur update of the ghost B at the low face of dim d
// (k_mur_low_b): Bg' = prev - i1m + kc (B1 - i1p - Bg + igm) + igp,
// prev' = B1.  lprev holds the adjoint of prev' on entry and of prev on
// exit; the laser's incident terms add their coefficient gradients to
// genv (one FP64 value per spline coefficient).
template <typename Real>
__global__ void k_mur_low_b_adj(GridInfo g, FieldPtrs<Real> l, int d, Real* lprev0,
                                Real* lprev1, LaserDev L, int64_t step, double* genv) {
  __shared__ double acc[64];
  for (int q = threadIdx.x; q < 64; q += blockDim.x) acc[q] = 0.0;
  __syncthreads();
  int a_dim = d == 0 ? 1 : 0, b_dim = d == 2 ? 1 : 2;
  int64_t np = (int64_t)g.n[a_dim] * g.n[b_dim];
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < 2 * np) {
    int q = (int)(t / np);
    int64_t pi = t % np;
    int a, b, na;
    face_ab(g, d, pi, a, b, na);
    int comp = q == 0 ? (d == 0 ? 1 : 0) : (d == 2 ? 1 : 2);
    Real* lB = l.B[comp];
    Real* lprev = q == 0 ? lprev0 : lprev1;
    const double kc = (g.dt - g.dx[d]) / (g.dt + g.dx[d]);
    const int64_t fg = face_node(g, d, -1, a, b), f1 = face_node(g, d, 0, a, b);
    const double lg = (double)lB[fg];
    const double lp_new = (double)lprev[pi];
    lprev[pi] = (Real)lg;
    lB[f1] = (Real)((double)lB[f1] + kc * lg + lp_new);
    lB[fg] = (Real)(-kc * lg);
    if (d == 0 && L.on && L.n_env > 0 && lg != 0.0) {
      const double tn = (double)step * g.dt;
      const int jj = a, kk = b;
      b_incident_grad(g, L, comp, -1, jj, kk, tn + 0.5 * g.dt, lg, acc);
      b_incident_grad(g, L, comp, -1, jj, kk, tn - 0.5 * g.dt, kc * lg, acc);
      b_incident_grad(g, L, comp, 0, jj, kk, tn - 0.5 * g.dt, -lg, acc);
      b_incident_grad(g, L, comp, 0, jj, kk, tn + 0.5 * g.dt, -kc * lg, acc);
    }
  }
  __syncthreads();
  if (d == 0 && L.on && L.n_env > 0)
    for (int q = threadIdx.x; q < L.n_env; q += blockDim.x)
      if (acc[q] != 0.0) atomicAdd(&genv[q], acc[q]);
}

// Transpose of saving the tangential E of the last interior layer.
template <typename Real>
__global__ void k_save_high_e_adj(GridInfo g, FieldPtrs<Real> l, int d, Real* ls0, Real* ls1) {
  int a_dim = d == 0 ? 1 : 0, b_dim = d == 2 ? 1 : 2;
  int64_t np = (int64_t)g.n[a_dim] * g.n[b_dim];
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * np) return;
  int q = (int)(t / np);
  int64_t pi = t % np;
  int a, b, na;
  face_ab(g, d, pi, a, b, na);
  int comp = q == 0 ? (d == 0 ? 1 : 0) : (d == 2 ? 1 : 2);
  Real* ls = q == 0 ? ls0 : ls1;
  const int64_t f1 = face_node(g, d, g.n[d] - 1, a, b);
  l.E[comp][f1] += ls[pi];
  ls[pi] = Real(0);
}

// Transpose of the Mur update of the ghost E at the high face of dim d
// (k_mur_high_e): Eg' = s + kc (E1 - Eg).
template <typename Real>
__global__ void k_mur_high_e_adj(GridInfo g, FieldPtrs<Real> l, int d, Real* ls0, Real* ls1) {
  int a_dim = d == 0 ? 1 : 0, b_dim = d == 2 ? 1 : 2;
  int64_t np = (int64_t)g.n[a_dim] * g.n[b_dim];
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * np) return;
  int q = (int)(t / np);
  int64_t pi = t % np;
  int a, b, na;
  face_ab(g, d, pi, a, b, na);
  int comp = q == 0 ? (d == 0 ? 1 : 0) : (d == 2 ? 1 : 2);
  Real* ls = q == 0 ? ls0 : ls1;
  const double kc = (g.dt - g.dx[d]) / (g.dt + g.dx[d]);
  Real* lE = l.E[comp];
  const int64_t fg = face_node(g, d, g.n[d], a, b), f1 = face_node(g, d, g.n[d] - 1, a, b);
  const double lg = (double)lE[fg];
  ls[pi] = (Real)lg;
  lE[f1] = (Real)((double)lE[f1] + kc * lg);
  lE[fg] = (Real)(-kc * lg);
}

// Adjoint of the probe recording of one step: l(field at probe p) +=
// cot[p * nsteps + rec].
template <typename Real>
__global__ void k_probe_seed(FieldPtrs<Real> l, int nprobe, const int* comp, const int64_t* index,
                             const double* cot, int64_t nsteps, int64_t rec) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nprobe) return;
  const int c = comp[p];
  Real* F = c < 3 ? l.E[c] : l.B[c - 3];
  const double v = cot[(int64_t)p * nsteps + rec];
  if (v != 0.0) atomicAdd(&F[index[p]], (Real)v);
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

template <typename Real>
void launch_zero(Real* p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  int64_t nb = (n + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_zero<Real>, dim3((unsigned)nb), 256, 0, st, p, n);
}

template <typename Real>
void launch_fill_periodic(const GridInfo& g, Real* const* comps, int ncomp, hipStream_t st,
                          bool reverse) {
  for (int it = 0; it < g.nd; it++) {
    const int d = reverse ? g.nd - 1 - it : it;
    if (!g.periodic[d]) continue;
    int a_dim = d == 0 ? 1 : 0, b_dim = d == 2 ? 1 : 2;
    int64_t total = (int64_t)g.st[a_dim] * g.st[b_dim] * 2 * kGuard;
    for (int c0 = 0; c0 < ncomp; c0 += 3) {
      int nc = ncomp - c0 < 3 ? ncomp - c0 : 3;
      hipLaunchKernelGGL(k_fill_periodic<Real>, blocks_for(total, 256), 256, 0, st, g, d,
                         comps[c0], nc > 1 ? comps[c0 + 1] : nullptr,
                         nc > 2 ? comps[c0 + 2] : nullptr, nc);
    }
  }
}

template <typename Real>
void launch_fold_periodic(const GridInfo& g, Real* const* comps, int ncomp, hipStream_t st,
                          bool reverse) {
  for (int it = 0; it < g.nd; it++) {
    const int d = reverse ? g.nd - 1 - it : it;
    if (!g.periodic[d]) continue;
    int a_dim = d == 0 ? 1 : 0, b_dim = d == 2 ? 1 : 2;
    int64_t total = (int64_t)g.st[a_dim] * g.st[b_dim] * 2 * kGuard;
    for (int c0 = 0; c0 < ncomp; c0 += 3) {
      int nc = ncomp - c0 < 3 ? ncomp - c0 : 3;
      hipLaunchKernelGGL(k_fold_periodic<Real>, blocks_for(total, 256), 256, 0, st, g, d,
                         comps[c0], nc > 1 ? comps[c0 + 1] : nullptr,
                         nc > 2 ? comps[c0 + 2] : nullptr, nc);
    }
  }
}

void launch_fold_periodic_f64(const GridInfo& g, double* rho, hipStream_t st) {
  double* c[1] = {rho};
  launch_fold_periodic<double>(g, c, 1, st, false);
}

template <typename Real>
void launch_b_half(const GridInfo& g, const FieldPtrs<Real>& f, hipStream_t st) {
  int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
  Real h = (Real)(0.5 * g.dt);
  Real ix = (Real)(1.0 / g.dx[0]);
  Real iy = g.nd > 1 ? (Real)(1.0 / g.dx[1]) : Real(0);
  Real iz = g.nd > 2 ? (Real)(1.0 / g.dx[2]) : Real(0);
  unsigned nb = blocks_for(ncell, 256);
  if (g.nd == 1) hipLaunchKernelGGL((k_b_half<Real, 1>), nb, 256, 0, st, g, f, h, ix, iy, iz);
  if (g.nd == 2) hipLaunchKernelGGL((k_b_half<Real, 2>), nb, 256, 0, st, g, f, h, ix, iy, iz);
  if (g.nd == 3) hipLaunchKernelGGL((k_b_half<Real, 3>), nb, 256, 0, st, g, f, h, ix, iy, iz);
}

template <typename Real>
void launch_e_full(const GridInfo& g, const FieldPtrs<Real>& f, hipStream_t st) {
  int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
  Real dt = (Real)g.dt;
  Real ix = (Real)(1.0 / g.dx[0]);
  Real iy = g.nd > 1 ? (Real)(1.0 / g.dx[1]) : Real(0);
  Real iz = g.nd > 2 ? (Real)(1.0 / g.dx[2]) : Real(0);
  unsigned nb = blocks_for(ncell, 256);
  if (g.nd == 1) hipLaunchKernelGGL((k_e_full<Real, 1>), nb, 256, 0, st, g, f, dt, ix, iy, iz);
  if (g.nd == 2) hipLaunchKernelGGL((k_e_full<Real, 2>), nb, 256, 0, st, g, f, dt, ix, iy, iz);
  if (g.nd == 3) hipLaunchKernelGGL((k_e_full<Real, 3>), nb, 256, 0, st, g, f, dt, ix, iy, iz);
}

template <typename Real, int ND>
static hipError_t launch_yee_fused_nd(const GridInfo& g, const FieldPtrs<Real>& fi,
                                      const FieldPtrs<Real>& fo, const MurHistory<Real>& mh,
                                      const LaserDev& las, int64_t step, hipStream_t st) {
  using T = YeeTile<Real, ND>;
  const int64_t ntiles = (int64_t)((g.n[0] + T::TX - 1) / T::TX) *
                         (ND > 1 ? (g.n[1] + T::TY - 1) / T::TY : 1);
  const Real h = (Real)(0.5 * g.dt), dt = (Real)g.dt;
  const Real ix = (Real)(1.0 / g.dx[0]);
  const Real iy = ND > 1 ? (Real)(1.0 / g.dx[1]) : Real(0);
  hipLaunchKernelGGL((k_yee_fused<Real, ND>), dim3((unsigned)ntiles), dim3(256), T::lds, st, g,
                     fi, fo, mh, las, step, h, dt, ix, iy);
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_yee_fused(const GridInfo& g, const FieldPtrs<Real>& fi, const FieldPtrs<Real>& fo,
                            Real* const hist_in[3][2], Real* const hist_out[3][2],
                            const LaserDev& las, int64_t step, hipStream_t st) {
  MurHistory<Real> mh{};
  for (int d = 0; d < 3; d++)
    for (int t = 0; t < 2; t++) {
      mh.in[d][t] = hist_in[d][t];
      mh.out[d][t] = hist_out[d][t];
    }
  if (g.nd == 1) return launch_yee_fused_nd<Real, 1>(g, fi, fo, mh, las, step, st);
  if (g.nd == 2) return launch_yee_fused_nd<Real, 2>(g, fi, fo, mh, las, step, st);
  return hipErrorInvalidValue;
}

static int64_t face_count(const GridInfo& g, int d) {
  int a_dim = d == 0 ? 1 : 0, b_dim = d == 2 ? 1 : 2;
  return (int64_t)g.n[a_dim] * g.n[b_dim];
}

template <typename Real>
void launch_mur_low_b(const GridInfo& g, const FieldPtrs<Real>& f, int d, Real* prev0,
                      Real* prev1, const LaserDev& las, int64_t step, hipStream_t st) {
  int64_t np = 2 * face_count(g, d);
  hipLaunchKernelGGL(k_mur_low_b<Real>, blocks_for(np, 256), 256, 0, st, g, f, d, prev0, prev1,
                     las, step);
}

template <typename Real>
void launch_save_high_e(const GridInfo& g, const FieldPtrs<Real>& f, int d, Real* s0, Real* s1,
                        hipStream_t st) {
  int64_t np = 2 * face_count(g, d);
  hipLaunchKernelGGL(k_save_high_e<Real>, blocks_for(np, 256), 256, 0, st, g, f, d, s0, s1);
}

template <typename Real>
void launch_mur_high_e(const GridInfo& g, const FieldPtrs<Real>& f, int d, const Real* s0,
                       const Real* s1, hipStream_t st) {
  int64_t np = 2 * face_count(g, d);
  hipLaunchKernelGGL(k_mur_high_e<Real>, blocks_for(np, 256), 256, 0, st, g, f, d, s0, s1);
}

template <typename Real>
void launch_probes(const GridInfo& g, const FieldPtrs<Real>& f, int nprobe, const int* comp,
                   const int64_t* index, Real* buf, int64_t max_steps, int64_t rec,
                   hipStream_t st) {
  if (nprobe <= 0 || rec >= max_steps) return;
  hipLaunchKernelGGL(k_probes<Real>, blocks_for(nprobe, 64), 64, 0, st, g, f, nprobe, comp, index,
                     buf, max_steps, rec);
}

template <typename Real>
static unsigned ext_blocks(const GridInfo& g) {
  int64_t n = (int64_t)(g.n[0] + 1) * (g.nd > 1 ? g.n[1] + 1 : 1) * (g.nd > 2 ? g.n[2] + 1 : 1);
  return blocks_for(n, 256);
}

template <typename Real>
void launch_b_half_adj(const GridInfo& g, const FieldPtrs<Real>& l, hipStream_t st) {
  Real h = (Real)(0.5 * g.dt);
  Real ix = (Real)(1.0 / g.dx[0]);
  Real iy = g.nd > 1 ? (Real)(1.0 / g.dx[1]) : Real(0);
  Real iz = g.nd > 2 ? (Real)(1.0 / g.dx[2]) : Real(0);
  unsigned nb = ext_blocks<Real>(g);
  if (g.nd == 1) hipLaunchKernelGGL((k_b_half_adj<Real, 1>), nb, 256, 0, st, g, l, h, ix, iy, iz);
  if (g.nd == 2) hipLaunchKernelGGL((k_b_half_adj<Real, 2>), nb, 256, 0, st, g, l, h, ix, iy, iz);
  if (g.nd == 3) hipLaunchKernelGGL((k_b_half_adj<Real, 3>), nb, 256, 0, st, g, l, h, ix, iy, iz);
}

template <typename Real>
void launch_e_full_adj(const GridInfo& g, const FieldPtrs<Real>& l, hipStream_t st) {
  Real dt = (Real)g.dt;
  Real ix = (Real)(1.0 / g.dx[0]);
  Real iy = g.nd > 1 ? (Real)(1.0 / g.dx[1]) : Real(0);
  Real iz = g.nd > 2 ? (Real)(1.0 / g.dx[2]) : Real(0);
  unsigned nb = ext_blocks<Real>(g);
  if (g.nd == 1) hipLaunchKernelGGL((k_e_full_adj<Real, 1>), nb, 256, 0, st, g, l, dt, ix, iy, iz);
  if (g.nd == 2) hipLaunchKernelGGL((k_e_full_adj<Real, 2>), nb, 256, 0, st, g, l, dt, ix, iy, iz);
  if (g.nd == 3) hipLaunchKernelGGL((k_e_full_adj<Real, 3>), nb, 256, 0, st, g, l, dt, ix, iy, iz);
}

template <typename Real>
void launch_mur_low_b_adj(const GridInfo& g, const FieldPtrs<Real>& l, int d, Real* lprev0,
                          Real* lprev1, const LaserDev& las, int64_t step, double* genv,
                          hipStream_t st) {
  int64_t np = 2 * face_count(g, d);
  hipLaunchKernelGGL(k_mur_low_b_adj<Real>, blocks_for(np, 256), 256, 0, st, g, l, d, lprev0,
                     lprev1, las, step, genv);
}

template <typename Real>
void launch_save_high_e_adj(const GridInfo& g, const FieldPtrs<Real>& l, int d, Real* ls0,
                            Real* ls1, hipStream_t st) {
  int64_t np = 2 * face_count(g, d);
  hipLaunchKernelGGL(k_save_high_e_adj<Real>, blocks_for(np, 256), 256, 0, st, g, l, d, ls0, ls1);
}

template <typename Real>
void launch_mur_high_e_adj(const GridInfo& g, const FieldPtrs<Real>& l, int d, Real* ls0,
                           Real* ls1, hipStream_t st) {
  int64_t np = 2 * face_count(g, d);
  hipLaunchKernelGGL(k_mur_high_e_adj<Real>, blocks_for(np, 256), 256, 0, st, g, l, d, ls0, ls1);
}

template <typename Real>
void launch_probe_seed(const FieldPtrs<Real>& l, int nprobe, const int* comp,
                       const int64_t* index, const double* cot, int64_t nsteps, int64_t rec,
                       hipStream_t st) {
  if (nprobe <= 0) return;
  hipLaunchKernelGGL(k_probe_seed<Real>, blocks_for(nprobe, 64), 64, 0, st, l, nprobe, comp,
                     index, cot, nsteps, rec);
}

#define PIC_INST(R)                                                                              \
  template void launch_zero<R>(R*, int64_t, hipStream_t);                                        \
  template void launch_fill_periodic<R>(const GridInfo&, R* const*, int, hipStream_t, bool);     \
  template void launch_fold_periodic<R>(const GridInfo&, R* const*, int, hipStream_t, bool);     \
  template void launch_b_half<R>(const GridInfo&, const FieldPtrs<R>&, hipStream_t);             \
  template void launch_e_full<R>(const GridInfo&, const FieldPtrs<R>&, hipStream_t);             \
  template void launch_mur_low_b<R>(const GridInfo&, const FieldPtrs<R>&, int, R*, R*,           \
                                    const LaserDev&, int64_t, hipStream_t);                      \
  template void launch_save_high_e<R>(const GridInfo&, const FieldPtrs<R>&, int, R*, R*,         \
                                      hipStream_t);                                              \
  template void launch_mur_high_e<R>(const GridInfo&, const FieldPtrs<R>&, int, const R*,        \
                                     const R*, hipStream_t);                                     \
  template hipError_t launch_yee_fused<R>(const GridInfo&, const FieldPtrs<R>&,                 \
                                          const FieldPtrs<R>&, R* const[3][2], R* const[3][2],   \
                                          const LaserDev&, int64_t, hipStream_t);                \
  template void launch_probes<R>(const GridInfo&, const FieldPtrs<R>&, int, const int*,          \
                                 const int64_t*, R*, int64_t, int64_t, hipStream_t);                   \
  template void launch_b_half_adj<R>(const GridInfo&, const FieldPtrs<R>&, hipStream_t);         \
  template void launch_e_full_adj<R>(const GridInfo&, const FieldPtrs<R>&, hipStream_t);         \
  template void launch_mur_low_b_adj<R>(const GridInfo&, const FieldPtrs<R>&, int, R*, R*,       \
                                        const LaserDev&, int64_t, double*, hipStream_t);         \
  template void launch_save_high_e_adj<R>(const GridInfo&, const FieldPtrs<R>&, int, R*, R*,     \
                                          hipStream_t);                                          \
  template void launch_mur_high_e_adj<R>(const GridInfo&, const FieldPtrs<R>&, int, R*, R*,      \
                                         hipStream_t);                                           \
  template void launch_probe_seed<R>(const FieldPtrs<R>&, int, const int*, const int64_t*,       \
                                     const double*, int64_t, int64_t, hipStream_t);

PIC_INST(float)
PIC_INST(double)

}  // namespace pic
