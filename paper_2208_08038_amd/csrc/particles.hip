// particles.hip -- the particle cycle with fields read from the guarded Yee
// planes in HBM and the current scattered with hardware floating-point
// atomics.  Used where a tile's field and current patches do not fit in
// LDS, and as the reference launch of the tiled kernel's arithmetic.
//
// One lane advances one macro-particle through the whole cycle; the state
// is read once and written once (structure of arrays, coalesced).
#include "cycle.h"

namespace pic {

namespace {

template <typename Real, int ND, bool TWO>
__global__ void __launch_bounds__(256) k_push(GridInfo g, FieldPtrs<Real> f, SpeciesDev<Real> s,
                                              PushConst<Real> c, uint32_t* err) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= s.n) return;
  PState<Real> st;
  load_state<Real, ND, TWO>(s, c, p, st);
  int ci[3];
  decode_cell<ND>(g, st.cell, ci);
  const int base = (int)g.origin + ci[0] + ci[1] * (int)g.sy + ci[2] * (int)g.sz;
  advance_particle<Real, ND, TWO, true>(g, s, c, p, st, ci, f, base, (int)g.sy, (int)g.sz, f.J,
                                        base, (int)g.sy, (int)g.sz, err);
}

// Particles listed by the tiled kernel (outside their tile since the last
// sort): advanced from HBM, current added with global atomics.  Runs after
// every colour of the tiled kernel of the species has finished.
template <typename Real, int ND, bool TWO>
__global__ void __launch_bounds__(256) k_push_list(GridInfo g, FieldPtrs<Real> f,
                                                   SpeciesDev<Real> s, PushConst<Real> c,
                                                   const uint32_t* list, const uint32_t* count,
                                                   uint32_t* total, uint32_t* err) {
  const uint32_t n = *count;
  if (blockIdx.x == 0 && threadIdx.x == 0 && n) atomicAdd(total, n);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    int64_t p = list[i];
    PState<Real> st;
    load_state<Real, ND, TWO>(s, c, p, st);
    int ci[3];
    decode_cell<ND>(g, st.cell, ci);
    const int base = (int)g.origin + ci[0] + ci[1] * (int)g.sy + ci[2] * (int)g.sz;
    advance_particle<Real, ND, TWO, true>(g, s, c, p, st, ci, f, base, (int)g.sy, (int)g.sz,
                                          f.J, base, (int)g.sy, (int)g.sz, err);
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

template <typename Real>
void launch_push_list(const GridInfo& g, const FieldPtrs<Real>& f, const SpeciesDev<Real>& s,
                      const PushConst<Real>& c, const uint32_t* list, const uint32_t* count,
                      uint32_t* total, uint32_t* err, hipStream_t st) {
  if (s.n == 0) return;
  dim3 grid(512), block(256);
  if (c.two_body) {
    if (g.nd == 1) hipLaunchKernelGGL((k_push_list<Real, 1, true>), grid, block, 0, st, g, f, s, c, list, count, total, err);
    if (g.nd == 2) hipLaunchKernelGGL((k_push_list<Real, 2, true>), grid, block, 0, st, g, f, s, c, list, count, total, err);
    if (g.nd == 3) hipLaunchKernelGGL((k_push_list<Real, 3, true>), grid, block, 0, st, g, f, s, c, list, count, total, err);
  } else {
    if (g.nd == 1) hipLaunchKernelGGL((k_push_list<Real, 1, false>), grid, block, 0, st, g, f, s, c, list, count, total, err);
    if (g.nd == 2) hipLaunchKernelGGL((k_push_list<Real, 2, false>), grid, block, 0, st, g, f, s, c, list, count, total, err);
    if (g.nd == 3) hipLaunchKernelGGL((k_push_list<Real, 3, false>), grid, block, 0, st, g, f, s, c, list, count, total, err);
  }
}

template void launch_push_list<float>(const GridInfo&, const FieldPtrs<float>&,
                                      const SpeciesDev<float>&, const PushConst<float>&,
                                      const uint32_t*, const uint32_t*, uint32_t*, uint32_t*,
                                      hipStream_t);
template void launch_push_list<double>(const GridInfo&, const FieldPtrs<double>&,
                                       const SpeciesDev<double>&, const PushConst<double>&,
                                       const uint32_t*, const uint32_t*, uint32_t*, uint32_t*,
                                       hipStream_t);

template void launch_push<float>(const GridInfo&, const FieldPtrs<float>&,
                                 const SpeciesDev<float>&, const PushConst<float>&, uint32_t*,
                                 hipStream_t);
template void launch_push<double>(const GridInfo&, const FieldPtrs<double>&,
                                  const SpeciesDev<double>&, const PushConst<double>&, uint32_t*,
                                  hipStream_t);

}  // namespace pic
