// load.h -- device-side particle loading (FP64 device arrays -> state).
#pragma once

#include "pic_internal.h"

namespace pic {

// FP64 device arrays of one load call (layout as in pic_load_particles).
struct LoadSrc {
  const double* x;
  const double* delta;
  const double* u1;
  const double* u2;
  const double* wc;
  const double* w;
  int64_t n;
};

struct LoadSplit {
  double q1, m1, q2, m2;
  double omega_c, weight;  // species defaults for the optional per-particle arrays
};

template <typename Real>
void launch_load(const GridInfo& g, const LoadSrc& src, const SpeciesDev<Real>& s, int64_t at,
                 int64_t* ids, const LoadSplit& sp, bool two, uint32_t* err, hipStream_t st);
// err: 16 bytes, zeroed by the caller: [0] error bits (PIC_ERR_*), bytes
// 8..15 the bits of the largest |weight| loaded (a non-negative double).

}  // namespace pic
