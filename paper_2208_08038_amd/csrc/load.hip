// load.hip -- conversion of FP64 particle arrays already resident in device
// memory into the library's state: position -> (packed cell, offset in the
// working precision), Sec. 2 momentum split of a centre-of-mass momentum,
// range checks.  Mirrors the host loader's arithmetic operation for
// operation (x / dx, floor, subtraction, rounding, crossing rule).
#include "pic_internal.h"
#include "load.h"

namespace pic {

namespace {

// Sec. 2 split: m1 u1 + m2 u2 = m_c u_c, q1 v1 + q2 v2 = 0 (see the host
// loader for the derivation); safeguarded Newton iteration on the speed of
// body 2.
__device__ void split_dev(double q1, double m1, double q2, double m2, const double uc[3],
                          double u1[3], double u2[3]) {
  double mc = m1 + m2;
  double p = sqrt(uc[0] * uc[0] + uc[1] * uc[1] + uc[2] * uc[2]);
  if (p == 0.0) {
    for (int a = 0; a < 3; a++) u1[a] = u2[a] = 0.0;
    return;
  }
  if (q1 + q2 == 0.0) {
    for (int a = 0; a < 3; a++) u1[a] = u2[a] = uc[a];
    return;
  }
  double al = -q2 / q1;
  double smax = fabs(al) > 1.0 ? 1.0 / fabs(al) : 1.0;
  double target = mc * p;
  double lo = 0.0, hi = smax;
  double s = fmin(target / (m1 * al + m2), 0.5 * smax);
  for (int it = 0; it < 100; it++) {
    double g1 = 1.0 / sqrt(1.0 - al * al * s * s), g2 = 1.0 / sqrt(1.0 - s * s);
    double gval = m1 * al * s * g1 + m2 * s * g2 - target;
    if (gval < 0)
      lo = s;
    else
      hi = s;
    double dg = m1 * al * g1 * g1 * g1 + m2 * g2 * g2 * g2;
    double sn = s - gval / dg;
    if (!(sn > lo && sn < hi)) sn = 0.5 * (lo + hi);
    if (sn == s) break;
    s = sn;
  }
  double g2 = 1.0 / sqrt(1.0 - s * s);
  double g1 = 1.0 / sqrt(1.0 - al * al * s * s);
  for (int a = 0; a < 3; a++) {
    double e = uc[a] / p;
    u2[a] = g2 * s * e;
    u1[a] = g1 * al * s * e;
  }
}

template <typename Real, int ND, bool TWO>
__global__ void __launch_bounds__(256) k_load(GridInfo g, LoadSrc src, SpeciesDev<Real> s,
                                              int64_t at, int64_t* ids, LoadSplit sp,
                                              uint32_t* err) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= src.n) return;
  int64_t q = at + p;
  uint32_t bad = 0;
  int ci[3] = {0, 0, 0};
  Real offr[3] = {0, 0, 0};
#pragma unroll
  for (int d = 0; d < ND; d++) {
    double xv = src.x[p * ND + d];
    if (!isfinite(xv)) {
      bad |= PIC_ERR_NAN;
      continue;
    }
    double xi = xv / g.dx[d];
    double f = floor(xi);
    if (f < 0.0 || f >= (double)g.n[d]) {
      bad |= PIC_ERR_RANGE;
      continue;
    }
    int c = (int)f;
    double o = xi - f;
    if (!g.periodic[d]) {
      double pos = f + o;
      if (pos < (double)g.pad || pos > (double)(g.n[d] - g.pad)) bad |= PIC_ERR_RANGE;
    }
    Real orr = (Real)o;
    if (orr >= Real(1)) {
      orr -= Real(1);
      c += 1;
      if (c >= g.n[d]) {
        if (g.periodic[d])
          c -= g.n[d];
        else
          bad |= PIC_ERR_RANGE;
      }
    }
    ci[d] = c;
    offr[d] = orr;
  }
  double u1[3], u2[3] = {0, 0, 0}, dl[3] = {0, 0, 0};
  for (int a = 0; a < 3; a++) {
    u1[a] = src.u1[3 * p + a];
    if (!isfinite(u1[a])) bad |= PIC_ERR_NAN;
  }
  if constexpr (TWO) {
    if (src.u2) {
      for (int a = 0; a < 3; a++) {
        u2[a] = src.u2[3 * p + a];
        if (!isfinite(u2[a])) bad |= PIC_ERR_NAN;
      }
    } else if (!bad) {
      double uc[3] = {u1[0], u1[1], u1[2]};
      split_dev(sp.q1, sp.m1, sp.q2, sp.m2, uc, u1, u2);
    }
    const double mc = sp.m1 + sp.m2;
    for (int a = 0; a < 3; a++) {
      dl[a] = src.delta ? src.delta[3 * p + a] : 0.0;
      if (!isfinite(dl[a])) bad |= PIC_ERR_NAN;
      // along walled axes each body lies between the walls
      if (a < ND && !g.periodic[a] && !bad) {
        const double X = src.x[p * ND + a] / g.dx[a];
        const double X1 = X + (sp.m2 / mc) * dl[a] / g.dx[a];
        const double X2 = X - (sp.m1 / mc) * dl[a] / g.dx[a];
        const double lo = g.pad, hi = g.n[a] - g.pad;
        if (!(X1 >= lo && X1 <= hi && X2 >= lo && X2 <= hi)) bad |= PIC_ERR_RANGE;
      }
    }
    if (src.wc && !(src.wc[p] > 0.0)) bad |= PIC_ERR_RANGE;
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
  for (int a = 0; a < 3; a++) s.u1[a][q] = (Real)u1[a];
  if constexpr (TWO) {
#pragma unroll
    for (int a = 0; a < 3; a++) {
      s.u2[a][q] = (Real)u2[a];
      s.dl[a][q] = (Real)dl[a];
    }
  }
  if (s.wc) s.wc[q] = (Real)(src.wc ? src.wc[p] : sp.omega_c);
  if (s.w) {
    const double w = src.w ? src.w[p] : sp.weight;
    s.w[q] = (Real)w;
    // largest |weight| of the load (bit order of non-negative doubles is
    // their numeric order), in bytes 8..15 of the error buffer
    atomicMax(reinterpret_cast<unsigned long long*>(err + 2),
              __builtin_bit_cast(unsigned long long, fabs(w)));
  }
  if (ids) ids[q] = q;
}

}  // namespace

template <typename Real>
void launch_load(const GridInfo& g, const LoadSrc& src, const SpeciesDev<Real>& s, int64_t at,
                 int64_t* ids, const LoadSplit& sp, bool two, uint32_t* err, hipStream_t st) {
  if (src.n <= 0) return;
  dim3 grid((unsigned)((src.n + 255) / 256));
  if (two) {
    if (g.nd == 1) hipLaunchKernelGGL((k_load<Real, 1, true>), grid, 256, 0, st, g, src, s, at, ids, sp, err);
    if (g.nd == 2) hipLaunchKernelGGL((k_load<Real, 2, true>), grid, 256, 0, st, g, src, s, at, ids, sp, err);
    if (g.nd == 3) hipLaunchKernelGGL((k_load<Real, 3, true>), grid, 256, 0, st, g, src, s, at, ids, sp, err);
  } else {
    if (g.nd == 1) hipLaunchKernelGGL((k_load<Real, 1, false>), grid, 256, 0, st, g, src, s, at, ids, sp, err);
    if (g.nd == 2) hipLaunchKernelGGL((k_load<Real, 2, false>), grid, 256, 0, st, g, src, s, at, ids, sp, err);
    if (g.nd == 3) hipLaunchKernelGGL((k_load<Real, 3, false>), grid, 256, 0, st, g, src, s, at, ids, sp, err);
  }
}

template void launch_load<float>(const GridInfo&, const LoadSrc&, const SpeciesDev<float>&,
                                 int64_t, int64_t*, const LoadSplit&, bool, uint32_t*,
                                 hipStream_t);
template void launch_load<double>(const GridInfo&, const LoadSrc&, const SpeciesDev<double>&,
                                  int64_t, int64_t*, const LoadSplit&, bool, uint32_t*,
                                  hipStream_t);

}  // namespace pic
