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

__device__ __forceinline__ double laser_time(const LaserDev& L, double tau) {
  if (tau < 0.0 || tau > L.t_env) return 0.0;
  double s = sin(3.14159265358979323846 * tau / L.t_env);
  return L.a0 * s * s * sin(L.omega * tau + L.phase);
}

// incident B of the laser (wave along +x) for component a at interior
// index (i, j, k) with the B stagger of that component
__device__ __forceinline__ double b_incident(const GridInfo& g, const LaserDev& L, int a, int i,
                                             int j, int k, double t) {
  if (!L.on) return 0.0;
  int want = L.pol == 2 ? 1 : 2;
  if (a != want) return 0.0;
  // B_a is half-staggered along the two axes other than a
  double sx = 0.5, sy = a == 1 ? 0.0 : 0.5, sz = a == 2 ? 0.0 : 0.5;
  double x = ((double)i + sx) * g.dx[0];
  if (L.oblique) {
    // plane wave travelling at an angle toward +y: B = n x E (c = 1), so the
    // in-plane E gives B_z = |E| and E_z gives B_y = -cos(angle) E_z
    double y = g.nd > 1 ? ((double)j + sy) * g.dx[1] - L.yc : 0.0;
    double e = laser_time(L, t - L.t_delay - (x * L.cos_a + y * L.sin_a));
    return a == 2 ? e : -L.cos_a * e;
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
  double e = prof * laser_time(L, t - L.t_delay - x);
  return a == 2 ? e : -e;
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

template <typename Real>
__global__ void k_probes(GridInfo g, FieldPtrs<Real> f, int nprobe, const int* comp,
                         const int64_t* index, Real* buf, int64_t max_steps, int64_t rec) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nprobe) return;
  int c = comp[p];
  const Real* F = c < 3 ? f.E[c] : f.B[c - 3];
  buf[(int64_t)p * max_steps + rec] = F[index[p]];
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
void launch_fill_periodic(const GridInfo& g, Real* const* comps, int ncomp, hipStream_t st) {
  for (int d = 0; d < g.nd; d++) {
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
void launch_fold_periodic(const GridInfo& g, Real* const* comps, int ncomp, hipStream_t st) {
  for (int d = 0; d < g.nd; d++) {
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
  launch_fold_periodic<double>(g, c, 1, st);
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

#define PIC_INST(R)                                                                              \
  template void launch_zero<R>(R*, int64_t, hipStream_t);                                        \
  template void launch_fill_periodic<R>(const GridInfo&, R* const*, int, hipStream_t);           \
  template void launch_fold_periodic<R>(const GridInfo&, R* const*, int, hipStream_t);           \
  template void launch_b_half<R>(const GridInfo&, const FieldPtrs<R>&, hipStream_t);             \
  template void launch_e_full<R>(const GridInfo&, const FieldPtrs<R>&, hipStream_t);             \
  template void launch_mur_low_b<R>(const GridInfo&, const FieldPtrs<R>&, int, R*, R*,           \
                                    const LaserDev&, int64_t, hipStream_t);                      \
  template void launch_save_high_e<R>(const GridInfo&, const FieldPtrs<R>&, int, R*, R*,         \
                                      hipStream_t);                                              \
  template void launch_mur_high_e<R>(const GridInfo&, const FieldPtrs<R>&, int, const R*,        \
                                     const R*, hipStream_t);                                     \
  template void launch_probes<R>(const GridInfo&, const FieldPtrs<R>&, int, const int*,          \
                                 const int64_t*, R*, int64_t, int64_t, hipStream_t);

PIC_INST(float)
PIC_INST(double)

}  // namespace pic
