// diag.hip -- FP64 diagnostics: charge density, charge-continuity residual,
// field and kinetic energy, total momentum.
//
// Sums are compensated (Neumaier) in FP64 even when the particle state and
// fields are FP32.  A fixed grid of REDUCE_BLOCKS blocks strides over the
// data, each block reduces its lanes in a fixed tree, and one final block
// adds the block partials in index order, so results are reproducible
// run to run.
#include "pic_internal.h"

namespace pic {

namespace {

constexpr int REDUCE_BLOCKS = 1024;
constexpr int RB = 256;

struct KSum {
  double s, c;
};

__device__ __forceinline__ void kadd(KSum& a, double v) {
  double t = a.s + v;
  if (fabs(a.s) >= fabs(v))
    a.c += (a.s - t) + v;
  else
    a.c += (v - t) + a.s;
  a.s = t;
}

__device__ __forceinline__ KSum kmerge(KSum a, KSum b) {
  kadd(a, b.s);
  a.c += b.c;
  return a;
}

// Block reduction of K compensated sums; thread 0 writes them to out[k*nb + block].
template <int K>
__device__ void block_reduce(KSum (&v)[K], double* out, int nb) {
  __shared__ double ss[K][RB], sc[K][RB];
  int t = threadIdx.x;
  for (int k = 0; k < K; k++) {
    ss[k][t] = v[k].s;
    sc[k][t] = v[k].c;
  }
  __syncthreads();
  for (int w = RB / 2; w > 0; w >>= 1) {
    if (t < w) {
      for (int k = 0; k < K; k++) {
        KSum a{ss[k][t], sc[k][t]}, b{ss[k][t + w], sc[k][t + w]};
        KSum m = kmerge(a, b);
        ss[k][t] = m.s;
        sc[k][t] = m.c;
      }
    }
    __syncthreads();
  }
  if (t == 0)
    for (int k = 0; k < K; k++) {
      out[(2 * k) * nb + blockIdx.x] = ss[k][0];
      out[(2 * k + 1) * nb + blockIdx.x] = sc[k][0];
    }
}

// final: out[k] = sum over blocks of partials (compensated); kind[k] = 1 for a max
__global__ void k_final(const double* partials, int nb, int K, int max_mask, double* out) {
  __shared__ double ss[RB], sc[RB];
  for (int k = 0; k < K; k++) {
    int t = threadIdx.x;
    bool mx = ((max_mask >> k) & 1) != 0;
    KSum acc{0.0, 0.0};
    double m = 0.0;
    for (int b = t; b < nb; b += RB) {
      double s = partials[(2 * k) * nb + b], c = partials[(2 * k + 1) * nb + b];
      if (mx) {
        m = fmax(m, s);
      } else {
        acc = kmerge(acc, KSum{s, c});
      }
    }
    ss[t] = mx ? m : acc.s;
    sc[t] = mx ? 0.0 : acc.c;
    __syncthreads();
    for (int w = RB / 2; w > 0; w >>= 1) {
      if (t < w) {
        if (mx) {
          ss[t] = fmax(ss[t], ss[t + w]);
        } else {
          KSum r = kmerge(KSum{ss[t], sc[t]}, KSum{ss[t + w], sc[t + w]});
          ss[t] = r.s;
          sc[t] = r.c;
        }
      }
      __syncthreads();
    }
    if (t == 0) out[k] = mx ? ss[0] : ss[0] + sc[0];
    __syncthreads();
  }
}

__device__ __forceinline__ void interior_ijk(const GridInfo& g, int64_t t, int& i, int& j, int& k) {
  i = (int)(t % g.n[0]);
  int64_t r = t / g.n[0];
  j = (int)(r % g.n[1]);
  k = (int)(r / g.n[1]);
}

template <typename Real>
__global__ void __launch_bounds__(RB) k_field_energy(GridInfo g, FieldPtrs<Real> f,
                                                     double* partials) {
  KSum v[1] = {{0.0, 0.0}};
  int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
  for (int64_t t = (int64_t)blockIdx.x * RB + threadIdx.x; t < ncell;
       t += (int64_t)gridDim.x * RB) {
    int i, j, k;
    interior_ijk(g, t, i, j, k);
    int64_t o = g.origin + i + j * g.sy + k * g.sz;
    double s = 0.0;
    for (int a = 0; a < 3; a++) {
      double e = f.E[a][o], b = f.B[a][o];
      s += e * e + b * b;
    }
    kadd(v[0], s);
  }
  block_reduce<1>(v, partials, gridDim.x);
}

template <typename Real>
__global__ void __launch_bounds__(RB) k_kinetic(SpeciesDev<Real> s, PushConst<Real> c,
                                                double* partials) {
  KSum v[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
  double m1 = c.m1, m2 = c.m2;
  for (int64_t p = (int64_t)blockIdx.x * RB + threadIdx.x; p < s.n; p += (int64_t)gridDim.x * RB) {
    double W = s.w ? (double)s.w[p] : (double)c.weight;
    double u[3], e = 0;
    double uu = 0;
    for (int q = 0; q < 3; q++) {
      u[q] = s.u1[q][p];
      uu += u[q] * u[q];
    }
    e += W * m1 * (sqrt(1.0 + uu) - 1.0);
    double pm[3] = {W * m1 * u[0], W * m1 * u[1], W * m1 * u[2]};
    if (c.two_body) {
      uu = 0;
      for (int q = 0; q < 3; q++) {
        u[q] = s.u2[q][p];
        uu += u[q] * u[q];
      }
      e += W * m2 * (sqrt(1.0 + uu) - 1.0);
      for (int q = 0; q < 3; q++) pm[q] += W * m2 * u[q];
    }
    kadd(v[0], e);
    for (int q = 0; q < 3; q++) kadd(v[1 + q], pm[q]);
  }
  block_reduce<4>(v, partials, gridDim.x);
}

// charge density at integer nodes: both bodies (or the point particle)
// with the quadratic B-spline, FP64 atomics into a guarded FP64 plane; each
// body in the frame of the cell that holds it (wrapped along periodic
// axes), so bodies may be any distance from their centre of mass
template <typename Real, int ND>
__global__ void __launch_bounds__(256) k_rho(GridInfo g, SpeciesDev<Real> s, PushConst<Real> c,
                                             double* rho) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= s.n) return;
  uint32_t packed = s.cell[p];
  int ci[3];
  ci[0] = packed & ((1u << g.bits[0]) - 1u);
  ci[1] = ND > 1 ? (packed >> g.bits[0]) & ((1u << g.bits[1]) - 1u) : 0;
  ci[2] = ND > 2 ? (packed >> (g.bits[0] + g.bits[1])) : 0;
  double dv = 1.0;
  for (int d = 0; d < ND; d++) dv *= g.dx[d];
  double W = s.w ? (double)s.w[p] : 1.0;
  int nb = c.two_body ? 2 : 1;
  for (int body = 0; body < nb; body++) {
    double Q = s.w ? (body == 0 ? (double)c.q1 : (double)c.q2) * W
                   : (body == 0 ? (double)c.qw1 : (double)c.qw2);
    double x[3] = {0, 0, 0};
    bool ok = true;
    for (int d = 0; d < ND; d++) {
      double o = s.off[d][p];
      if (c.two_body) {
        double sd = (double)s.dl[d][p] * (double)c.idx[d];
        x[d] = body == 0 ? o + (double)c.f1 * sd : o - (double)c.f2 * sd;
      } else {
        x[d] = o;
      }
      ok = ok && isfinite(x[d]);
    }
    if (ok) rho_add_body<ND>(g, ci, x, Q, dv, rho);
  }
}

// Charge density of a tile-sorted species: one workgroup per tile adds the
// bodies of its sorted range into an FP64 LDS patch covering the tile's
// cells with two nodes around them (the nodes of every body in its cell
// and of any body within one cell of it), then adds each non-zero patch
// node to the plane with one global atomic.  A body whose nodes leave the
// patch (a particle that drifted since the sort, a far body) or the
// guarded plane's interior [-2, n + 1] goes straight to the plane as in
// k_rho.  Same sum as k_rho up to the order of the FP64 adds.
template <typename Real, int ND>
__global__ void __launch_bounds__(256) k_rho_tiled(GridInfo g, SpeciesDev<Real> s,
                                                   PushConst<Real> c, const uint32_t* tile_off,
                                                   TileGrid t, double* rho) {
  extern __shared__ double patch[];
  const int64_t tile = blockIdx.x;
  const int64_t p0 = tile_off[tile], p1 = tile_off[tile + 1];
  if (p0 == p1) return;  // the whole block leaves before any barrier
  int lo[3] = {0, 0, 0}, P[3] = {1, 1, 1};
  int64_t r = tile;
  for (int d = 0; d < ND; d++) {
    const int tc = (int)(r % t.nt[d]);
    r /= t.nt[d];
    lo[d] = tc * t.T[d] - 2;
    P[d] = t.T[d] + 4;
  }
  const int np = P[0] * P[1] * P[2];
  for (int q = threadIdx.x; q < np; q += blockDim.x) patch[q] = 0.0;
  __syncthreads();
  double dv = 1.0;
  for (int d = 0; d < ND; d++) dv *= g.dx[d];
  const int nb = c.two_body ? 2 : 1;
  for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
    const uint32_t packed = s.cell[p];
    int ci[3];
    ci[0] = packed & ((1u << g.bits[0]) - 1u);
    ci[1] = ND > 1 ? (packed >> g.bits[0]) & ((1u << g.bits[1]) - 1u) : 0;
    ci[2] = ND > 2 ? (packed >> (g.bits[0] + g.bits[1])) : 0;
    const double W = s.w ? (double)s.w[p] : 1.0;
    for (int body = 0; body < nb; body++) {
      const double Q = s.w ? (body == 0 ? (double)c.q1 : (double)c.q2) * W
                           : (body == 0 ? (double)c.qw1 : (double)c.qw2);
      double x[3] = {0, 0, 0};
      bool ok = true;
      for (int d = 0; d < ND; d++) {
        const double o = s.off[d][p];
        if (c.two_body) {
          const double sd = (double)s.dl[d][p] * (double)c.idx[d];
          x[d] = body == 0 ? o + (double)c.f1 * sd : o - (double)c.f2 * sd;
        } else {
          x[d] = o;
        }
        ok = ok && isfinite(x[d]);
      }
      if (!ok) continue;
      // first of the three nodes along each axis (unwrapped node index),
      // its index in the patch, and the weights
      int a[3] = {0, 0, 0};
      double w[3][3] = {{1, 0, 0}, {1, 0, 0}, {1, 0, 0}};
      bool in = true;
      for (int d = 0; d < ND; d++) {
        const double k = floor(x[d]);
        const double xf = x[d] - k;
        const double f = floor(xf + 0.5), dd = xf - f;
        const int n0 = ci[d] + (int)k + (int)f - 1;
        a[d] = n0 - lo[d];
        in = in && a[d] >= 0 && a[d] + 2 < P[d] && n0 >= -2 && n0 + 2 <= g.n[d] + 1;
        w[d][0] = 0.5 * (0.5 - dd) * (0.5 - dd);
        w[d][1] = 0.75 - dd * dd;
        w[d][2] = 0.5 * (0.5 + dd) * (0.5 + dd);
      }
      if (!in) {
        rho_add_body<ND>(g, ci, x, Q, dv, rho);
        continue;
      }
      const double qv = Q / dv;
      const int nz = ND > 2 ? 3 : 1, ny = ND > 1 ? 3 : 1;
      for (int cz = 0; cz < nz; cz++)
        for (int cy = 0; cy < ny; cy++)
          for (int cx = 0; cx < 3; cx++) {
            const double wt = w[0][cx] * w[1][cy] * w[2][cz];
            const int q = (a[0] + cx) + P[0] * ((a[1] + cy) + P[1] * (a[2] + cz));
            if (wt != 0.0) atomicAdd(patch + q, qv * wt);
          }
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < np; q += blockDim.x) {
    const double v = patch[q];
    if (v == 0.0) continue;
    const int i = lo[0] + q % P[0];
    const int j = lo[1] + (q / P[0]) % P[1];
    const int k = lo[2] + q / (P[0] * P[1]);
    unsafeAtomicAdd(rho + g.origin + i + (int64_t)j * g.sy + (int64_t)k * g.sz, v);
  }
}

// residual (rho1 - rho0)/dt + div J at every interior node
template <typename Real>
__global__ void __launch_bounds__(RB) k_residual(GridInfo g, FieldPtrs<Real> f, const double* rho0,
                                                 const double* rho1, double* partials) {
  KSum v[3] = {{0, 0}, {0, 0}, {0, 0}};
  double mx = 0.0;
  int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
  for (int64_t t = (int64_t)blockIdx.x * RB + threadIdx.x; t < ncell;
       t += (int64_t)gridDim.x * RB) {
    int ijk[3];
    interior_ijk(g, t, ijk[0], ijk[1], ijk[2]);
    int64_t o = g.origin + ijk[0] + ijk[1] * g.sy + ijk[2] * g.sz;
    double drho = (rho1[o] - rho0[o]) / g.dt;
    double div = 0.0;
    for (int d = 0; d < g.nd; d++) {
      int64_t sd = d == 0 ? 1 : (d == 1 ? g.sy : g.sz);
      double jm = 0.0;
      if (g.periodic[d]) {
        int64_t om = ijk[d] == 0 ? o + (int64_t)(g.n[d] - 1) * sd : o - sd;
        jm = f.J[d][om];
      } else if (ijk[d] > 0) {
        jm = f.J[d][o - sd];
      }
      div += ((double)f.J[d][o] - jm) / g.dx[d];
    }
    double r = drho + div;
    kadd(v[0], r * r);
    kadd(v[2], drho * drho);
    mx = fmax(mx, fabs(r));
  }
  // the maximum is reduced on its own and stored in slot 1 of the partials
  __shared__ double smax[RB];
  smax[threadIdx.x] = mx;
  __syncthreads();
  for (int w = RB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
    __syncthreads();
  }
  double bmax = smax[0];
  __syncthreads();
  v[1].s = 0.0;
  block_reduce<3>(v, partials, gridDim.x);
  if (threadIdx.x == 0) {
    partials[2 * gridDim.x + blockIdx.x] = bmax;
    partials[3 * gridDim.x + blockIdx.x] = 0.0;
  }
}

}  // namespace

int reduce_blocks() { return REDUCE_BLOCKS; }

// max_mask: bit k set when quantity k is a maximum rather than a sum
static void final_reduce(double* partials, int nb, int K, int max_mask, double* out,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_final, 1, RB, 0, st, partials, nb, K, max_mask, out);
}

template <typename Real>
void launch_field_energy(const GridInfo& g, const FieldPtrs<Real>& f, double* partials, int nb,
                         double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_field_energy<Real>, nb, RB, 0, st, g, f, partials);
  final_reduce(partials, nb, 1, 0, out, st);
}

template <typename Real>
void launch_kinetic(const SpeciesDev<Real>& s, const PushConst<Real>& c, double* partials, int nb,
                    double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_kinetic<Real>, nb, RB, 0, st, s, c, partials);
  final_reduce(partials, nb, 4, 0, out, st);
}

template <typename Real>
void launch_rho(const GridInfo& g, const SpeciesDev<Real>& s, const PushConst<Real>& c,
                double* rho, hipStream_t st) {
  if (s.n == 0) return;
  unsigned nb = (unsigned)((s.n + 255) / 256);
  if (g.nd == 1) hipLaunchKernelGGL((k_rho<Real, 1>), nb, 256, 0, st, g, s, c, rho);
  if (g.nd == 2) hipLaunchKernelGGL((k_rho<Real, 2>), nb, 256, 0, st, g, s, c, rho);
  if (g.nd == 3) hipLaunchKernelGGL((k_rho<Real, 3>), nb, 256, 0, st, g, s, c, rho);
}

size_t rho_tiled_lds(const GridInfo& g, const TileGrid& t) {
  size_t lds = sizeof(double);
  for (int d = 0; d < g.nd; d++) lds *= (size_t)(t.T[d] + 4);
  return lds;
}

template <typename Real>
void launch_rho_tiled(const GridInfo& g, const SpeciesDev<Real>& s, const PushConst<Real>& c,
                      const uint32_t* tile_off, const TileGrid& t, double* rho, hipStream_t st) {
  if (s.n == 0) return;
  if (rho_tiled_lds(g, t) > kRhoTiledMaxLds) {  // a patch this large: one thread per particle
    launch_rho<Real>(g, s, c, rho, st);
    return;
  }
  int64_t ntiles = 1;
  const size_t lds = rho_tiled_lds(g, t);
  for (int d = 0; d < g.nd; d++) ntiles *= t.nt[d];
  if (g.nd == 1)
    hipLaunchKernelGGL((k_rho_tiled<Real, 1>), dim3((unsigned)ntiles), 256, lds, st, g, s, c,
                       tile_off, t, rho);
  if (g.nd == 2)
    hipLaunchKernelGGL((k_rho_tiled<Real, 2>), dim3((unsigned)ntiles), 256, lds, st, g, s, c,
                       tile_off, t, rho);
  if (g.nd == 3)
    hipLaunchKernelGGL((k_rho_tiled<Real, 3>), dim3((unsigned)ntiles), 256, lds, st, g, s, c,
                       tile_off, t, rho);
}

template <typename Real>
void launch_residual(const GridInfo& g, const FieldPtrs<Real>& f, const double* rho0,
                     const double* rho1, double* partials, int nb, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_residual<Real>, nb, RB, 0, st, g, f, rho0, rho1, partials);
  final_reduce(partials, nb, 3, 2, out, st);
}

#define PIC_DIAG_INST(R)                                                                        \
  template void launch_field_energy<R>(const GridInfo&, const FieldPtrs<R>&, double*, int,      \
                                       double*, hipStream_t);                                   \
  template void launch_kinetic<R>(const SpeciesDev<R>&, const PushConst<R>&, double*, int,      \
                                  double*, hipStream_t);                                        \
  template void launch_rho<R>(const GridInfo&, const SpeciesDev<R>&, const PushConst<R>&,       \
                              double*, hipStream_t);                                            \
  template void launch_rho_tiled<R>(const GridInfo&, const SpeciesDev<R>&, const PushConst<R>&, \
                                    const uint32_t*, const TileGrid&, double*, hipStream_t);    \
  template void launch_residual<R>(const GridInfo&, const FieldPtrs<R>&, const double*,         \
                                   const double*, double*, int, double*, hipStream_t);

PIC_DIAG_INST(float)
PIC_DIAG_INST(double)

}  // namespace pic
