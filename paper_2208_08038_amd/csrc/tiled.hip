// tiled.hip -- the particle cycle, one workgroup per tile of cells.
//
// Particles are grouped by tile (tile sort).  A workgroup
//   1. stages E and B of its tile plus a 2-node apron into LDS,
//   2. clears an LDS current patch covering the tile plus the 2-node
//      (below) / 3-node (above) reach of the order-2 Esirkepov window,
//   3. advances every particle of the tile, gathering from LDS and
//      depositing with LDS floating-point atomics,
//   4. adds the patch into the global current with plain loads and stores.
// Tiles are launched in 2^ndim colours (parity of the tile coordinates):
// patches of tiles of one colour never overlap (patch extent T + 5 <= 2T),
// so step 4 needs no global atomics and the sum order is fixed.  A
// particle that has drifted out of its tile since the last sort is only
// listed here; a second kernel advances the listed particles from HBM
// after the last colour, adding their current with global atomics.
#include "cycle.h"
#include "tiled.h"

namespace pic {

namespace {

// The LDS current patch accumulates in FP64 whatever the working precision:
// on gfx950 FP32 LDS atomic adds issue far slower than FP64 ones (measured
// with SQ_WAIT_INST_LDS), and the wider sum also drops the rounding of the
// per-tile reduction.
using PatchT = double;

template <typename Real, int ND, bool TWO>
__device__ __forceinline__ void tiled_body(const GridInfo& g, const FieldPtrs<Real>& f,
                                           const SpeciesDev<Real>& s, const PushConst<Real>& c,
                                           const TileGeom& t, const uint32_t* tile_off, int color,
                                           uint32_t* list, uint32_t* nlist, uint32_t* err) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // tile of this block within the colour
  int b = blockIdx.x;
  int tc[3] = {0, 0, 0};
  tc[0] = 2 * (b % t.nc[0]) + (color & 1);
  b /= t.nc[0];
  if (ND > 1) {
    tc[1] = 2 * (b % t.nc[1]) + ((color >> 1) & 1);
    b /= t.nc[1];
  }
  if (ND > 2) tc[2] = 2 * b + ((color >> 2) & 1);
  for (int d = 0; d < ND; d++)
    if (tc[d] >= t.nt[d]) return;  // whole block leaves before any barrier
  int lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
  for (int d = 0; d < ND; d++) {
    lo[d] = tc[d] * t.T[d];
    hi[d] = min(lo[d] + t.T[d], g.n[d]);
  }
  const int64_t tile = tc[0] + (int64_t)t.nt[0] * (tc[1] + (int64_t)t.nt[1] * tc[2]);
  const int64_t p0 = tile_off[tile], p1 = tile_off[tile + 1];

  // LDS layout: E[3], B[3] on the field patch, then J[3] on the current patch
  const int FX = t.F[0], FY = t.F[1], FZ = t.F[2];
  const int JX = t.Jd[0], JY = t.Jd[1], JZ = t.Jd[2];
  const int nf = FX * FY * FZ, nj = JX * JY * JZ;
  FieldPtrs<Real> fl;
  PatchT* jl[3];
  // the FP64 patch comes first (8-byte aligned), the fields after it
  PatchT* pbase = reinterpret_cast<PatchT*>(smem_raw);
  Real* fbase_l = reinterpret_cast<Real*>(pbase + 3 * nj);
  for (int a = 0; a < 3; a++) {
    jl[a] = pbase + a * nj;
    fl.E[a] = fbase_l + a * nf;
    fl.B[a] = fbase_l + (3 + a) * nf;
    fl.J[a] = nullptr;
  }
  // patch origins in storage: field patch starts 2 nodes below the tile,
  // current patch likewise (it extends 3 nodes above)
  int64_t forg = g.origin;
  for (int d = 0; d < ND; d++) {
    int64_t sd = d == 0 ? 1 : (d == 1 ? g.sy : g.sz);
    forg += (int64_t)(lo[d] - 2) * sd;
  }
  // 1-2. stage fields (only the part a partial tile needs), clear the patch
  int fext[3] = {1, 1, 1};
  for (int d = 0; d < ND; d++) fext[d] = (hi[d] - lo[d]) + 4;
  for (int q = threadIdx.x; q < nf; q += blockDim.x) {
    int a = q % FX, r = q / FX;
    int bb = r % FY, cc = r / FY;
    if (a >= fext[0] || bb >= fext[1] || cc >= fext[2]) continue;
    int64_t go = forg + a + (int64_t)bb * g.sy + (int64_t)cc * g.sz;
#pragma unroll
    for (int comp = 0; comp < 3; comp++) {
      fl.E[comp][q] = f.E[comp][go];
      fl.B[comp][q] = f.B[comp][go];
    }
  }
  for (int q = threadIdx.x; q < 3 * nj; q += blockDim.x) jl[0][q] = PatchT(0);
  __syncthreads();

  // 3. particles of the tile
  const int fsy = FX, fsz = FX * FY;
  const int jsy = JX, jsz = JX * JY;
  const int lane = threadIdx.x & 63;
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  for (int64_t p0w = p0; p0w < p1; p0w += blockDim.x) {
    const int64_t p = p0w + threadIdx.x;
    const bool valid = p < p1;
    int ci[3] = {0, 0, 0};
    bool inside = false;
    if (valid) {
      decode_cell<ND>(g, s.cell[p], ci);
      inside = true;
#pragma unroll
      for (int d = 0; d < ND; d++) inside = inside && ci[d] >= lo[d] && ci[d] < hi[d];
    }
    // list the particles outside the tile: one atomic per wavefront
    const bool out = valid && !inside;
    const uint64_t m = __ballot(out);
    if (m) {
      uint32_t basei = 0;
      const int leader = __ffsll((unsigned long long)m) - 1;
      if (lane == leader) basei = atomicAdd(nlist, (uint32_t)__popcll(m));
      basei = __shfl(basei, leader);
      if (out) list[basei + (uint32_t)__popcll(m & below)] = (uint32_t)p;
    }
    if (valid && inside) {
      int lf = (ci[0] - lo[0] + 2);
      int lj = lf;
      if (ND > 1) {
        lf += (ci[1] - lo[1] + 2) * fsy;
        lj += (ci[1] - lo[1] + 2) * jsy;
      }
      if (ND > 2) {
        lf += (ci[2] - lo[2] + 2) * fsz;
        lj += (ci[2] - lo[2] + 2) * jsz;
      }
      advance_particle<Real, ND, TWO, false, PatchT>(g, s, c, p, ci, fl, lf, fsy, fsz, jl, lj,
                                                     jsy, jsz, err);
    }
  }
  __syncthreads();

  // 4. add the current patch into the global planes (no other tile of this
  //    colour touches these nodes)
  int64_t jorg = g.origin;
  int jext[3] = {1, 1, 1};
  for (int d = 0; d < ND; d++) {
    int64_t sd = d == 0 ? 1 : (d == 1 ? g.sy : g.sz);
    jorg += (int64_t)(lo[d] - 2) * sd;
    jext[d] = (hi[d] - lo[d]) + 5;
  }
  for (int q = threadIdx.x; q < nj; q += blockDim.x) {
    int a = q % JX, r = q / JX;
    int bb = r % JY, cc = r / JY;
    if (a >= jext[0] || bb >= jext[1] || cc >= jext[2]) continue;
    int64_t go = jorg + a + (int64_t)bb * g.sy + (int64_t)cc * g.sz;
#pragma unroll
    for (int comp = 0; comp < 3; comp++) {
      PatchT v = jl[comp][q];
      if (v != PatchT(0)) f.J[comp][go] = (Real)((PatchT)f.J[comp][go] + v);
    }
  }
}

// FP32 fields with the FP64 current patch of an 8^3 tile take 94 KB of LDS
// (one workgroup per CU); FP64 fields take 136 KB.  With one workgroup of
// 8 waves per CU each wave may use up to 256 VGPRs.
template <int ND, bool TWO>
__global__ void __launch_bounds__(kTiledThreads) __attribute__((amdgpu_waves_per_eu(2)))
k_push_tiled_f32(GridInfo g, FieldPtrs<float> f, SpeciesDev<float> s, PushConst<float> c,
                 TileGeom t, const uint32_t* tile_off, int color, uint32_t* list,
                 uint32_t* nlist, uint32_t* err) {
  tiled_body<float, ND, TWO>(g, f, s, c, t, tile_off, color, list, nlist, err);
}

template <int ND, bool TWO>
__global__ void __launch_bounds__(kTiledThreads) __attribute__((amdgpu_waves_per_eu(2)))
k_push_tiled_f64(GridInfo g, FieldPtrs<double> f, SpeciesDev<double> s, PushConst<double> c,
                 TileGeom t, const uint32_t* tile_off, int color, uint32_t* list,
                 uint32_t* nlist, uint32_t* err) {
  tiled_body<double, ND, TWO>(g, f, s, c, t, tile_off, color, list, nlist, err);
}

}  // namespace

TileGeom make_tile_geom(const GridInfo& g, const int tile[3], const int ntiles[3]) {
  TileGeom t{};
  for (int d = 0; d < 3; d++) {
    bool r = d < g.nd;
    t.T[d] = r ? tile[d] : 1;
    t.nt[d] = r ? ntiles[d] : 1;
    t.nc[d] = r ? (ntiles[d] + 1) / 2 : 1;
    t.F[d] = r ? tile[d] + 4 : 1;
    t.Jd[d] = r ? tile[d] + 5 : 1;
  }
  return t;
}

size_t tiled_lds_bytes(const TileGeom& t, size_t rsize) {
  size_t nf = (size_t)t.F[0] * t.F[1] * t.F[2];
  size_t nj = (size_t)t.Jd[0] * t.Jd[1] * t.Jd[2];
  return 6 * nf * rsize + 3 * nj * sizeof(double);
}

bool tiled_supported(const GridInfo& g, const TileGeom& t, size_t rsize) {
  for (int d = 0; d < g.nd; d++)
    if (t.T[d] < 5) return false;  // patches of same-colour tiles must not overlap
  return tiled_lds_bytes(t, rsize) <= kTiledMaxLds;
}

template <typename Real, int ND, bool TWO>
static hipError_t launch_colour(const GridInfo& g, const FieldPtrs<Real>& f,
                                const SpeciesDev<Real>& s, const PushConst<Real>& c,
                                const TileGeom& t, const uint32_t* tile_off, int color,
                                uint32_t* list, uint32_t* nlist, uint32_t* err, size_t lds,
                                hipStream_t st) {
  const void* fn;
  if constexpr (sizeof(Real) == 4)
    fn = (const void*)k_push_tiled_f32<ND, TWO>;
  else
    fn = (const void*)k_push_tiled_f64<ND, TWO>;
  static size_t attr_lds = 0;
  if (lds > 64 * 1024 && lds > attr_lds) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_lds = lds;
  }
  unsigned blocks = (unsigned)((int64_t)t.nc[0] * t.nc[1] * t.nc[2]);
  if constexpr (sizeof(Real) == 4)
    hipLaunchKernelGGL((k_push_tiled_f32<ND, TWO>), dim3(blocks), dim3(kTiledThreads), lds, st, g,
                       f, s, c, t, tile_off, color, list, nlist, err);
  else
    hipLaunchKernelGGL((k_push_tiled_f64<ND, TWO>), dim3(blocks), dim3(kTiledThreads), lds, st, g,
                       f, s, c, t, tile_off, color, list, nlist, err);
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_push_tiled(const GridInfo& g, const FieldPtrs<Real>& f, const SpeciesDev<Real>& s,
                             const PushConst<Real>& c, const TileGeom& t, const uint32_t* tile_off,
                             uint32_t* list, uint32_t* nlist, uint32_t* nlist_total,
                             uint32_t* err, hipStream_t st, DispatchHook hook) {
  if (s.n == 0) return hipSuccess;
  size_t lds = tiled_lds_bytes(t, sizeof(Real));
  hipError_t e = hipMemsetAsync(nlist, 0, sizeof(uint32_t), st);
  if (e != hipSuccess) return e;
  int ncol = 1 << g.nd;
  for (int color = 0; color < ncol; color++) {
    if (hook.fn) hook.fn(hook.arg, true);
    if (c.two_body) {
      if (g.nd == 1) e = launch_colour<Real, 1, true>(g, f, s, c, t, tile_off, color, list, nlist, err, lds, st);
      if (g.nd == 2) e = launch_colour<Real, 2, true>(g, f, s, c, t, tile_off, color, list, nlist, err, lds, st);
      if (g.nd == 3) e = launch_colour<Real, 3, true>(g, f, s, c, t, tile_off, color, list, nlist, err, lds, st);
    } else {
      if (g.nd == 1) e = launch_colour<Real, 1, false>(g, f, s, c, t, tile_off, color, list, nlist, err, lds, st);
      if (g.nd == 2) e = launch_colour<Real, 2, false>(g, f, s, c, t, tile_off, color, list, nlist, err, lds, st);
      if (g.nd == 3) e = launch_colour<Real, 3, false>(g, f, s, c, t, tile_off, color, list, nlist, err, lds, st);
    }
    if (e != hipSuccess) return e;
    if (hook.fn) hook.fn(hook.arg, false);
  }
  launch_push_list<Real>(g, f, s, c, list, nlist, nlist_total, err, st);
  return hipGetLastError();
}

template hipError_t launch_push_tiled<float>(const GridInfo&, const FieldPtrs<float>&,
                                             const SpeciesDev<float>&, const PushConst<float>&,
                                             const TileGeom&, const uint32_t*, uint32_t*,
                                             uint32_t*, uint32_t*, uint32_t*, hipStream_t,
                                             DispatchHook);
template hipError_t launch_push_tiled<double>(const GridInfo&, const FieldPtrs<double>&,
                                              const SpeciesDev<double>&, const PushConst<double>&,
                                              const TileGeom&, const uint32_t*, uint32_t*,
                                              uint32_t*, uint32_t*, uint32_t*, hipStream_t,
                                             DispatchHook);

}  // namespace pic
