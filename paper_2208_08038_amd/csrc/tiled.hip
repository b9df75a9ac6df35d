// tiled.hip -- the particle cycle, one workgroup per tile of cells.
//
// Particles are grouped by tile (tile sort).  A workgroup
//   1. stages E and B of its tile plus a 2-node apron into LDS,
//   2. clears an LDS current patch covering the tile plus the 2-node
//      (below) / 3-node (above) reach of the order-2 Esirkepov window,
//   3. advances every particle of the tile, gathering from LDS and
//      depositing with LDS atomics (64-bit fixed point for FP32 work, FP64
//      otherwise); a body whose nearest node changes needs the longer
//      four-node deposit, which is queued in LDS and run after the loop by
//      consecutive threads,
//   4. adds the patch into the global current with plain loads and stores.
// Tiles are launched in 2^ndim colours (parity of the tile coordinates):
// patches of tiles of one colour never overlap (patch extent T + 5 <= 2T),
// so step 4 needs no global atomics and the sum order is fixed.  A
// particle that has drifted out of its tile since the last sort is only
// listed here; a second kernel advances the listed particles from HBM
// after the last colour, adding their current with global atomics.
#include <algorithm>
#include <type_traits>

#include "cycle.h"
#include "tiled.h"

namespace pic {

namespace {

// LDS current patch: FP64 for FP64 work; for FP32 work 64-bit fixed point
// (exact, order-independent sums, and 64-bit integer LDS atomics issue
// faster than FP64 ones; FP32 LDS atomic adds issue slowest of all on
// gfx950).  The per-species scale keeps a term below 2^46 (host side; a
// shared patch takes the smaller of two species' scales), and a workgroup
// advances at most kChunk particles of each species (listing any further
// ones for the outside-tile kernel): at most 2^16 terms per node from the
// two bodies of the ions and 2^15 from a point species, below 2^63.
template <typename Real>
using PatchOf = std::conditional_t<sizeof(Real) == 4, long long, double>;
constexpr int64_t kChunk = 32768;

// LDS queue of general deposits (structure of arrays, `cap` entries).
template <typename Real, int ND>
struct LdsQueue {
  Real* val;        // queue_vals(ND) rows of cap values
  int* base;        // patch index of the body's cell
  uint32_t* count;  // entries requested (may exceed cap)
  int cap;
  __device__ __forceinline__ bool operator()(int jb, const Real* x0, const Real* x1, Real q,
                                             const Real* v) const {
    const uint32_t i = atomicAdd(count, 1u);
    if (i >= (uint32_t)cap) return false;  // full: the caller deposits at once
    base[i] = jb;
    int k = 0;
#pragma unroll
    for (int d = 0; d < ND; d++) val[(k++) * cap + i] = x0[d];
#pragma unroll
    for (int d = 0; d < ND; d++) val[(k++) * cap + i] = x1[d];
    val[(k++) * cap + i] = q;
#pragma unroll
    for (int d = ND; d < 3; d++) val[(k++) * cap + i] = v[d];
    return true;
  }
  __device__ __forceinline__ void load(int i, int& jb, Real x0[3], Real x1[3], Real& q,
                                       Real v[3]) const {
    jb = base[i];
    int k = 0;
#pragma unroll
    for (int d = 0; d < 3; d++) x0[d] = x1[d] = v[d] = Real(0);
#pragma unroll
    for (int d = 0; d < ND; d++) x0[d] = val[(k++) * cap + i];
#pragma unroll
    for (int d = 0; d < ND; d++) x1[d] = val[(k++) * cap + i];
    q = val[(k++) * cap + i];
#pragma unroll
    for (int d = ND; d < 3; d++) v[d] = val[(k++) * cap + i];
  }
};

// One species' share of a tiled launch: its particles, constants, tile
// offsets of its sorted order and its list of particles found outside
// their tile (with the list's counter).
template <typename Real>
struct TileSpecies {
  SpeciesDev<Real> s;
  PushConst<Real> c;
  const uint32_t* tile_off;
  uint32_t* list;
  uint32_t* nlist;
  uint32_t* nfar;  // two-body ions listed because their bodies are far apart
  // two-body ions whose bodies sit on different stencils are set aside
  // here (entry k of a tile at defer[p0 + k], p0 the tile's first sorted
  // particle) and advanced after the others; nullptr: advanced in place
  uint32_t* defer;
};

// Field and current patch indices of the node below the cell ci (the
// patches start two nodes below the tile's first cell lo).
template <int ND>
__device__ __forceinline__ void patch_bases(const int ci[3], const int lo[3], int fsy, int fsz,
                                            int jsy, int jsz, int& lf, int& lj) {
  lf = ci[0] - lo[0] + 2;
  lj = lf;
  if (ND > 1) {
    lf += (ci[1] - lo[1] + 2) * fsy;
    lj += (ci[1] - lo[1] + 2) * jsy;
  }
  if (ND > 2) {
    lf += (ci[2] - lo[2] + 2) * fsz;
    lj += (ci[2] - lo[2] + 2) * jsz;
  }
}

// 3. the particles [p0, p1) of one species in the tile; the state of a
//    thread's next particle is loaded while it advances the present one
//    (PREFETCH; costs the registers of one more state).  Beyond kChunk
//    particles (a tile far more crowded than the mean) the rest is listed
//    like particles outside the tile, which bounds the number of terms per
//    patch node.
//    Two-body ions whose bodies sit on different stencils take the
//    two-gather path; with sp.defer, a wavefront sets such ions aside and
//    advances them 64 at a time (all lanes on that path together) instead
//    of in the wavefront they were read in.  The j-th ion a wavefront sets
//    aside is kept at the j-th position of the tile range it has read
//    (position p0 + 64 w + (j / 64) nthr + j % 64 for its wave index w),
//    which no other wavefront reads or writes.
template <typename Real, int ND, bool TWO, bool PREFETCH>
__device__ __forceinline__ void tile_particles(const GridInfo& g, const TileSpecies<Real>& sp,
                                               int64_t p0, int64_t p1, const int lo[3],
                                               const int hi[3], const FieldPtrs<Real>& fl,
                                               int fsy, int fsz, PatchOf<Real>* const jl[3],
                                               int jsy, int jsz, const LdsQueue<Real, ND>& queue,
                                               uint32_t* err, int tid, int nthr) {
  using PatchT = PatchOf<Real>;
  const SpeciesDev<Real>& s = sp.s;
  const PushConst<Real>& c = sp.c;
  uint32_t* list = sp.list;
  uint32_t* nlist = sp.nlist;
  const int lane = threadIdx.x & 63;
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int64_t pk = p0 + kChunk;
  // set-aside slots of this wavefront: slot j at dbase + (j / 64) nthr + j % 64
  uint32_t* const dbase = TWO && sp.defer ? sp.defer + p0 + (tid - lane) : nullptr;
  uint32_t dput = 0, dget = 0;  // ions set aside / taken back (same in every lane)
  PState<Real> next;
  if (PREFETCH && p0 + tid < p1) load_state<Real, ND, TWO>(s, c, p0 + tid, next);
  int64_t p0w = p0;
  for (;;) {
    // a full batch of set-aside ions, or the last ones once the range is read
    const bool batch = TWO && dput > dget && (dput - dget >= 64u || p0w >= p1);
    if (!batch && p0w >= p1) break;
    int64_t p;
    bool valid;
    PState<Real> st;
    if (batch) {
      const uint32_t j = dget + (uint32_t)lane;
      valid = j < dput;
      p = valid ? (int64_t)dbase[(int64_t)(j >> 6) * nthr + (j & 63u)] : p1;
      if (valid) load_state<Real, ND, TWO>(s, c, p, st);
      dget = min(dget + 64u, dput);
    } else {
      p = p0w + tid;
      valid = p < p1;
      if (PREFETCH) {
        st = next;
        if (p + nthr < p1) load_state<Real, ND, TWO>(s, c, p + nthr, next);
      } else if (valid) {
        load_state<Real, ND, TWO>(s, c, p, st);
      }
      p0w += nthr;
    }
    int ci[3] = {0, 0, 0};
    bool inside = false, far = false, split = false;
    if (valid) {
      decode_cell<ND>(g, st.cell, ci);
      inside = p < pk;
#pragma unroll
      for (int d = 0; d < ND; d++) inside = inside && ci[d] >= lo[d] && ci[d] < hi[d];
      // an ion with a body beyond [-1/2, 3/2) of its cell reaches beyond the
      // tile's patches: the HBM pass takes it (each body in its own frame)
      if constexpr (TWO) {
        Real xa[3] = {0, 0, 0}, xb[3] = {0, 0, 0};
#pragma unroll
        for (int d = 0; d < ND; d++) {
          const Real sd = st.dl[d] * c.idx[d];
          xa[d] = st.off[d] + c.f1 * sd;
          xb[d] = st.off[d] - c.f2 * sd;
          far = far || !(body_near(xa[d]) && body_near(xb[d]));
        }
        split = !same_stencil<Real, ND>(xa, xb);
      }
    }
    // list the particles outside the tile: one atomic per wavefront (an ion
    // taken back from the set-aside slots was inside and near when read)
    const bool out = valid && (!inside || far);
    const uint64_t m = __ballot(out);
    if (m) {
      uint32_t basei = 0;
      const int leader = __ffsll((unsigned long long)m) - 1;
      if (lane == leader) basei = atomicAdd(nlist, (uint32_t)__popcll(m));
      basei = __shfl(basei, leader);
      if (out) list[basei + (uint32_t)__popcll(m & below)] = (uint32_t)p;
      if constexpr (TWO) {
        const uint64_t mf = __ballot(valid && far);
        if (mf && lane == leader) atomicAdd(sp.nfar, (uint32_t)__popcll(mf));
      }
    }
    bool go = valid && inside && !far;
    if constexpr (TWO) {
      if (dbase && !batch) {
        const bool aside = go && split;
        const uint64_t md = __ballot(aside);
        if (aside) {
          const uint32_t j = dput + (uint32_t)__popcll(md & below);
          dbase[(int64_t)(j >> 6) * nthr + (j & 63u)] = (uint32_t)p;
          go = false;
        }
        dput += (uint32_t)__popcll(md);
      }
    }
    if (go) {
      int lf, lj;
      patch_bases<ND>(ci, lo, fsy, fsz, jsy, jsz, lf, lj);
      advance_particle<Real, ND, TWO, false, PatchT>(g, s, c, p, st, ci, fl, lf, fsy, fsz, jl,
                                                     lj, jsy, jsz, err, queue);
    }
  }
}

// TX, TY, TZ > 0 fix the tile shape at compile time (patch strides become
// constants, so LDS addresses fold into instruction offsets); 0 takes the
// shape from `t`.  NS = 1: species `a` (two-body if TWO) alone.  NS = 2: a
// two-body species `a` and a point species `b` share the tile's staged
// fields and current patch (one staging and one flush for both), each
// advanced by its share of the workgroup's wavefronts; both species'
// constants carry the same fixed-point scale.
template <typename Real, int ND, bool TWO, int NS, int WPE, int TX, int TY, int TZ>
__device__ __forceinline__ void tiled_body(const GridInfo& g, const FieldPtrs<Real>& f,
                                           const TileSpecies<Real>& a, const TileSpecies<Real>& b,
                                           const TileGeom& t, int color, uint32_t* err) {
  static_assert(NS == 1 || TWO, "a shared launch pairs a two-body with a point species");
  using PatchT = PatchOf<Real>;
  const PushConst<Real>& c = a.c;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // tile of this block within the colour (from the occupied list in a
  // sparse launch).  Workgroups go round-robin over the 8 XCDs (each with
  // its own L2); consecutive tiles share cache lines of the field and
  // current planes, so in FP32 each XCD takes a contiguous run of them:
  // block b takes (b mod 8) B / 8 + min(b mod 8, B mod 8) + b / 8 of B
  // blocks (a quarter less HBM reading on the 3D slab).  The FP64 build,
  // with twice the particle bytes per tile, measured faster with tiles in
  // block order.
  int bi = blockIdx.x;
  if constexpr (sizeof(Real) == 4) {
    const int b = blockIdx.x, nb = gridDim.x, x = b & 7;
    bi = x * (nb >> 3) + min(x, nb & 7) + (b >> 3);
  }
  if (t.occ) {
    if ((uint32_t)bi >= t.occ[color]) return;
    bi = (int)t.occ[8 + (int64_t)color * ((int64_t)t.nc[0] * t.nc[1] * t.nc[2]) + bi];
  }
  int tc[3] = {0, 0, 0};
  tc[0] = 2 * (bi % t.nc[0]) + (color & 1);
  bi /= t.nc[0];
  if (ND > 1) {
    tc[1] = 2 * (bi % t.nc[1]) + ((color >> 1) & 1);
    bi /= t.nc[1];
  }
  if (ND > 2) tc[2] = 2 * bi + ((color >> 2) & 1);
  for (int d = 0; d < ND; d++)
    if (tc[d] >= t.nt[d]) return;  // whole block leaves before any barrier
  const int TT[3] = {TX ? TX : t.T[0], TY ? TY : t.T[1], TZ ? TZ : t.T[2]};
  int lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
  for (int d = 0; d < ND; d++) {
    lo[d] = tc[d] * TT[d];
    hi[d] = min(lo[d] + TT[d], g.n[d]);
  }
  const int64_t tile = tc[0] + (int64_t)t.nt[0] * (tc[1] + (int64_t)t.nt[1] * tc[2]);
  // a tile with no particle in its sorted range has nothing to stage,
  // advance or flush (the whole block leaves before any barrier)
  bool empty = a.tile_off[tile] == a.tile_off[tile + 1];
  if constexpr (NS == 2) empty = empty && b.tile_off[tile] == b.tile_off[tile + 1];
  if (empty) return;

  // LDS layout: the FP64 current patch first (8-byte aligned), then the
  // field pairs, then the deposit queue
  PatchLayout L;
  if constexpr (TX > 0) {
    constexpr PatchLayout Lc = patch_layout(TX, TY, TZ, ND);
    L = Lc;
  } else {
    L = t.L;
  }
  FieldPtrs<Real> fl;
  PatchT* jl[3];
  PatchT* pbase = reinterpret_cast<PatchT*>(smem_raw);
  Real* fbase_l = reinterpret_cast<Real*>(pbase + L.nj);
  for (int a = 0; a < 3; a++) {
    jl[a] = pbase + a * L.Jd[0];
    fl.J[a] = nullptr;
  }
  Real* fc[6];
  for (int cmp = 0; cmp < 6; cmp++) fc[cmp] = fbase_l + (cmp >> 1) * L.fpair + (cmp & 1) * L.F[0];
  for (int a = 0; a < 3; a++) {
    fl.E[a] = fc[a];
    fl.B[a] = fc[3 + a];
  }
  LdsQueue<Real, ND> queue;
  queue.cap = t.qcap;
  queue.val = fbase_l + 3 * L.fpair;
  queue.base = reinterpret_cast<int*>(queue.val + queue_vals(ND) * t.qcap);
  queue.count = reinterpret_cast<uint32_t*>(queue.base + t.qcap);
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
  const int nf = L.F[0] * L.F[1] * L.F[2];
  for (int q = threadIdx.x; q < nf; q += blockDim.x) {
    int a = q % L.F[0], r = q / L.F[0];
    int bb = r % L.F[1], cc = r / L.F[1];
    if (a >= fext[0] || bb >= fext[1] || cc >= fext[2]) continue;
    int64_t go = forg + a + (int64_t)bb * g.sy + (int64_t)cc * g.sz;
    const int li = a + bb * L.fpitch + cc * L.fplane;
#pragma unroll
    for (int comp = 0; comp < 3; comp++) {
      fl.E[comp][li] = f.E[comp][go];
      fl.B[comp][li] = f.B[comp][go];
    }
  }
  for (int q = threadIdx.x; q < L.nj; q += blockDim.x) pbase[q] = PatchT(0);
  if (threadIdx.x == 0) *queue.count = 0u;
  __syncthreads();

  const int fsy = L.fpitch, fsz = L.fplane;
  const int jsy = L.jpitch, jsz = L.jplane;
  constexpr bool PREFETCH_A = WPE < 4 || !TWO;
  const int64_t a0 = a.tile_off[tile], a1 = a.tile_off[tile + 1];
  if constexpr (NS == 1) {
    tile_particles<Real, ND, TWO, PREFETCH_A>(g, a, a0, a1, lo, hi, fl, fsy, fsz, jl, jsy, jsz,
                                              queue, err, threadIdx.x, blockDim.x);
  } else {
    // the wavefronts split between the species in proportion to their
    // work in this tile (an ion costs about 1.7 electrons), so that the
    // ions' arithmetic and the electrons' LDS traffic run side by side
    const int64_t b0 = b.tile_off[tile], b1 = b.tile_off[tile + 1];
    const int nw = (int)blockDim.x / 64;
    const double wi = 1.7 * (double)(a1 - a0), we = (double)(b1 - b0);
    int wa = wi + we > 0.0 ? (int)(nw * wi / (wi + we) + 0.5) : nw;
    if (a1 > a0 && b1 > b0) wa = min(max(wa, 1), nw - 1);
    const int split = 64 * wa;
    if ((int)threadIdx.x < split)
      tile_particles<Real, ND, true, PREFETCH_A>(g, a, a0, a1, lo, hi, fl, fsy, fsz, jl, jsy, jsz,
                                                 queue, err, threadIdx.x, split);
    else
      tile_particles<Real, ND, false, true>(g, b, b0, b1, lo, hi, fl, fsy, fsz, jl, jsy, jsz,
                                            queue, err, threadIdx.x - split,
                                            (int)blockDim.x - split);
  }
  __syncthreads();

  // 3b. the queued general deposits, one per thread
  const int nq = min((int)*queue.count, t.qcap);
  for (int e = threadIdx.x; e < nq; e += blockDim.x) {
    int jb;
    Real x0[3], x1[3], v[3], q;
    queue.load(e, jb, x0, x1, q, v);
    if (!deposit<Real, ND, false, PatchT>(jl, jb, jsy, jsz, x0, x1, q, v, c))
      atomicOr(err, PIC_ERR_RANGE);
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
  const double inv_scale = std::is_integral<PatchT>::value ? 1.0 / (double)c.jscale : 1.0;
  const int njn = L.Jd[0] * L.Jd[1] * L.Jd[2];
  for (int q = threadIdx.x; q < njn; q += blockDim.x) {
    int a = q % L.Jd[0], r = q / L.Jd[0];
    int bb = r % L.Jd[1], cc = r / L.Jd[1];
    if (a >= jext[0] || bb >= jext[1] || cc >= jext[2]) continue;
    int64_t go = jorg + a + (int64_t)bb * g.sy + (int64_t)cc * g.sz;
    const int li = a + bb * L.jpitch + cc * L.jplane;
#pragma unroll
    for (int comp = 0; comp < 3; comp++) {
      PatchT v = jl[comp][li];
      if (v != PatchT(0)) f.J[comp][go] = (Real)((double)f.J[comp][go] + (double)v * inv_scale);
    }
  }
}

// FP32 fields with the FP64 current patch of an 8^3 tile take 94 KB of LDS
// (one workgroup of 8 waves per CU: each wave may use up to 256 VGPRs);
// an 8x8x6 tile takes under 80 KB, so two workgroups fit when each wave
// keeps to 128 VGPRs (WPE = 4 waves per SIMD).
template <int ND, bool TWO, int NS, int WPE, int TX, int TY, int TZ>
__global__ void __launch_bounds__(kTiledThreads) __attribute__((amdgpu_waves_per_eu(WPE)))
k_push_tiled_f32(GridInfo g, FieldPtrs<float> f, TileSpecies<float> a, TileSpecies<float> b,
                 TileGeom t, int color, uint32_t* err) {
  tiled_body<float, ND, TWO, NS, WPE, TX, TY, TZ>(g, f, a, b, t, color, err);
}

template <int ND, bool TWO, int NS, int WPE, int TX, int TY, int TZ>
__global__ void __launch_bounds__(kTiledThreads) __attribute__((amdgpu_waves_per_eu(WPE)))
k_push_tiled_f64(GridInfo g, FieldPtrs<double> f, TileSpecies<double> a, TileSpecies<double> b,
                 TileGeom t, int color, uint32_t* err) {
  tiled_body<double, ND, TWO, NS, WPE, TX, TY, TZ>(g, f, a, b, t, color, err);
}

}  // namespace

namespace {

struct OccSpecies {
  const uint32_t* tile_off[kOccSpecies];
  int n;
};

// One workgroup: count and list, per colour, the tiles whose sorted range
// is non-empty for some species.  Rounds of 1024 consecutive tiles; within a
// round each tile's place in its colour's list is the count of busy tiles
// of that colour before it (wave ballots, then the waves before), so the
// lists keep tile order.
__global__ void __launch_bounds__(1024) k_occupied_tiles(TileGeom t, OccSpecies sp, uint32_t* occ) {
  __shared__ uint32_t base[8];
  __shared__ uint32_t wcnt[16][8];
  if (threadIdx.x < 8) base[threadIdx.x] = 0;
  __syncthreads();
  const int64_t ntile = (int64_t)t.nt[0] * t.nt[1] * t.nt[2];
  const int64_t per_colour = (int64_t)t.nc[0] * t.nc[1] * t.nc[2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t below = (uint64_t(1) << lane) - 1;
  for (int64_t t0 = 0; t0 < ntile; t0 += 1024) {
    const int64_t tile = t0 + threadIdx.x;
    bool busy = false;
    int colour = 0;
    uint32_t bi = 0;
    if (tile < ntile) {
      for (int s = 0; s < sp.n; s++)
        busy = busy || sp.tile_off[s][tile] != sp.tile_off[s][tile + 1];
      const int tx = (int)(tile % t.nt[0]);
      const int ty = (int)((tile / t.nt[0]) % t.nt[1]);
      const int tz = (int)(tile / ((int64_t)t.nt[0] * t.nt[1]));
      colour = (tx & 1) | ((ty & 1) << 1) | ((tz & 1) << 2);
      bi = (uint32_t)((tx >> 1) + t.nc[0] * ((ty >> 1) + t.nc[1] * (tz >> 1)));
    }
    uint32_t rank = 0;
#pragma unroll
    for (int c = 0; c < 8; c++) {
      const uint64_t m = __ballot(busy && colour == c);
      if (lane == 0) wcnt[wave][c] = (uint32_t)__popcll(m);
      if (busy && colour == c) rank = (uint32_t)__popcll(m & below);
    }
    __syncthreads();
    if (busy) {
      uint32_t at = base[colour] + rank;
      for (int w = 0; w < wave; w++) at += wcnt[w][colour];
      occ[8 + colour * per_colour + at] = bi;
    }
    __syncthreads();
    if (threadIdx.x < 8) {
      uint32_t add = 0;
      for (int w = 0; w < 16; w++) add += wcnt[w][threadIdx.x];
      base[threadIdx.x] += add;
    }
    __syncthreads();
  }
  if (threadIdx.x < 8) occ[threadIdx.x] = base[threadIdx.x];
}

}  // namespace

hipError_t launch_occupied_tiles(const TileGeom& t, const uint32_t* const* tile_off, int nspecies,
                                 uint32_t* occ, hipStream_t st) {
  if (nspecies > kOccSpecies) return hipErrorInvalidValue;
  OccSpecies sp{};
  for (int s = 0; s < nspecies; s++) sp.tile_off[s] = tile_off[s];
  sp.n = nspecies;
  hipLaunchKernelGGL(k_occupied_tiles, dim3(1), dim3(1024), 0, st, t, sp, occ);
  return hipGetLastError();
}

TileGeom make_tile_geom(const GridInfo& g, const int tile[3], const int ntiles[3], size_t rsize) {
  TileGeom t{};
  t.nd = g.nd;
  for (int d = 0; d < 3; d++) {
    bool r = d < g.nd;
    t.T[d] = r ? tile[d] : 1;
    t.nt[d] = r ? ntiles[d] : 1;
    t.nc[d] = r ? (ntiles[d] + 1) / 2 : 1;
  }
  t.L = patch_layout(t.T[0], t.T[1], t.T[2], g.nd);
  // the queue takes what LDS is left, up to kQueueMax entries; when the
  // patches leave room for 32 entries within half the LDS, it stops there
  // so that two workgroups can share a CU (a full queue only sends the
  // overflow down the direct path)
  t.qcap = 0;
  size_t fixed = tiled_lds_bytes(t, rsize);
  size_t entry = (size_t)queue_vals(g.nd) * rsize + sizeof(int);
  size_t limit = fixed + 32 * entry <= kTiledMaxLds / 2 ? kTiledMaxLds / 2 : kTiledMaxLds;
  if (fixed < limit) {
    size_t room = (limit - fixed) / entry;
    t.qcap = (int)std::min<size_t>(room, kQueueMax) & ~15;
  }
  return t;
}

// patch, fields, queue (values, cell indices) and the queue counter
size_t tiled_lds_bytes(const TileGeom& t, size_t rsize) {
  size_t queue = (size_t)t.qcap * ((size_t)queue_vals(t.nd) * rsize + sizeof(int));
  return (size_t)t.L.nj * sizeof(double) + 3 * (size_t)t.L.fpair * rsize + queue + 16;
}

bool tiled_supported(const GridInfo& g, const TileGeom& t, size_t rsize) {
  for (int d = 0; d < g.nd; d++)
    if (t.T[d] < 5) return false;  // patches of same-colour tiles must not overlap
  return tiled_lds_bytes(t, rsize) <= kTiledMaxLds;
}

template <typename Real, int ND, bool TWO, int NS, int WPE, int TX, int TY, int TZ>
static const void* tiled_kernel() {
  if constexpr (sizeof(Real) == 4)
    return (const void*)k_push_tiled_f32<ND, TWO, NS, WPE, TX, TY, TZ>;
  else
    return (const void*)k_push_tiled_f64<ND, TWO, NS, WPE, TX, TY, TZ>;
}

template <typename Real, int ND, bool TWO, int NS, int WPE, int TX, int TY, int TZ>
static hipError_t launch_colour_wpe(const GridInfo& g, const FieldPtrs<Real>& f,
                                    const TileSpecies<Real>& a, const TileSpecies<Real>& b,
                                    const TileGeom& t, int color, uint32_t* err, size_t lds,
                                    hipStream_t st) {
  static size_t attr_lds = 0;
  if (lds > 64 * 1024 && lds > attr_lds) {
    hipError_t e = hipFuncSetAttribute(tiled_kernel<Real, ND, TWO, NS, WPE, TX, TY, TZ>(),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_lds = lds;
  }
  const int64_t per_colour = (int64_t)t.nc[0] * t.nc[1] * t.nc[2];
  unsigned blocks = (unsigned)(t.occ ? std::min<int64_t>(t.occ_n[color], per_colour) : per_colour);
  if (blocks == 0) return hipSuccess;
  if constexpr (sizeof(Real) == 4)
    hipLaunchKernelGGL((k_push_tiled_f32<ND, TWO, NS, WPE, TX, TY, TZ>), dim3(blocks),
                       dim3(kTiledThreads), lds, st, g, f, a, b, t, color, err);
  else
    hipLaunchKernelGGL((k_push_tiled_f64<ND, TWO, NS, WPE, TX, TY, TZ>), dim3(blocks),
                       dim3(kTiledThreads), lds, st, g, f, a, b, t, color, err);
  return hipGetLastError();
}

// True if the 4-waves-per-SIMD build of the kernel keeps everything in
// registers (no scratch).
template <typename Real, int ND, bool TWO, int NS, int TX, int TY, int TZ>
static bool wpe4_without_spill() {
  static int ok = -1;
  if (ok < 0) {
    hipFuncAttributes fa{};
    ok = hipFuncGetAttributes(&fa, tiled_kernel<Real, ND, TWO, NS, 4, TX, TY, TZ>()) ==
                     hipSuccess &&
                 fa.localSizeBytes == 0
             ? 1
             : 0;
  }
  return ok == 1;
}

// two workgroups per CU when their LDS fits and the smaller register
// budget needs no spills, else one with the larger register budget
template <typename Real, int ND, bool TWO, int NS, int TX, int TY, int TZ>
static hipError_t launch_colour_shape(const GridInfo& g, const FieldPtrs<Real>& f,
                                      const TileSpecies<Real>& a, const TileSpecies<Real>& b,
                                      const TileGeom& t, int color, uint32_t* err, size_t lds,
                                      hipStream_t st) {
  if (2 * lds <= kTiledMaxLds && wpe4_without_spill<Real, ND, TWO, NS, TX, TY, TZ>())
    return launch_colour_wpe<Real, ND, TWO, NS, 4, TX, TY, TZ>(g, f, a, b, t, color, err, lds, st);
  return launch_colour_wpe<Real, ND, TWO, NS, 2, TX, TY, TZ>(g, f, a, b, t, color, err, lds, st);
}

// the default tiles (3D: 8x8x6 for FP32, 8x8x8 for FP64; 2D: 12x12) have
// builds with compile-time strides; any other shape runs the generic build
template <typename Real, int ND, bool TWO, int NS>
static hipError_t launch_colour(const GridInfo& g, const FieldPtrs<Real>& f,
                                const TileSpecies<Real>& a, const TileSpecies<Real>& b,
                                const TileGeom& t, int color, uint32_t* err, size_t lds,
                                hipStream_t st) {
  if constexpr (ND == 3) {
    constexpr int TZ = sizeof(Real) == 4 ? 6 : 8;
    if (t.T[0] == 8 && t.T[1] == 8 && t.T[2] == TZ)
      return launch_colour_shape<Real, ND, TWO, NS, 8, 8, TZ>(g, f, a, b, t, color, err, lds, st);
  }
  if constexpr (ND == 2) {
    if (t.T[0] == 12 && t.T[1] == 12)
      return launch_colour_shape<Real, ND, TWO, NS, 12, 12, 1>(g, f, a, b, t, color, err, lds, st);
  }
  return launch_colour_shape<Real, ND, TWO, NS, 0, 0, 0>(g, f, a, b, t, color, err, lds, st);
}

template <typename Real, int NS>
static hipError_t launch_colours(const GridInfo& g, const FieldPtrs<Real>& f,
                                 const TileSpecies<Real>& a, const TileSpecies<Real>& b,
                                 const TileGeom& t, uint32_t* err, hipStream_t st,
                                 DispatchHook hook) {
  const size_t lds = tiled_lds_bytes(t, sizeof(Real));
  const bool two = NS == 2 || a.c.two_body;
  hipError_t e = hipSuccess;
  for (int color = 0; color < (1 << g.nd); color++) {
    if (hook.fn) hook.fn(hook.arg, true);
    if (two) {
      if (g.nd == 1) e = launch_colour<Real, 1, true, NS>(g, f, a, b, t, color, err, lds, st);
      if (g.nd == 2) e = launch_colour<Real, 2, true, NS>(g, f, a, b, t, color, err, lds, st);
      if (g.nd == 3) e = launch_colour<Real, 3, true, NS>(g, f, a, b, t, color, err, lds, st);
    } else if constexpr (NS == 1) {
      if (g.nd == 1) e = launch_colour<Real, 1, false, 1>(g, f, a, b, t, color, err, lds, st);
      if (g.nd == 2) e = launch_colour<Real, 2, false, 1>(g, f, a, b, t, color, err, lds, st);
      if (g.nd == 3) e = launch_colour<Real, 3, false, 1>(g, f, a, b, t, color, err, lds, st);
    }
    if (e != hipSuccess) return e;
    if (hook.fn) hook.fn(hook.arg, false);
  }
  return hipSuccess;
}

template <typename Real>
static TileSpecies<Real> tile_species(const SpeciesDev<Real>& s, const PushConst<Real>& c,
                                      const uint32_t* tile_off, uint32_t* list,
                                      uint32_t* nlist, uint32_t* nfar, uint32_t* defer) {
  return TileSpecies<Real>{s, c, tile_off, list, nlist, nfar, c.two_body ? defer : nullptr};
}

template <typename Real>
hipError_t launch_push_tiled(const GridInfo& g, const FieldPtrs<Real>& f, const SpeciesDev<Real>& s,
                             const PushConst<Real>& c, const TileGeom& t, const uint32_t* tile_off,
                             uint32_t* list, uint32_t* defer, uint32_t* nlist,
                             uint32_t* nlist_total, uint32_t* nfar, uint32_t* err, hipStream_t st,
                             DispatchHook hook) {
  if (s.n == 0) return hipSuccess;
  hipError_t e = hipMemsetAsync(nlist, 0, sizeof(uint32_t), st);
  if (e != hipSuccess) return e;
  const TileSpecies<Real> a = tile_species(s, c, tile_off, list, nlist, nfar, defer);
  e = launch_colours<Real, 1>(g, f, a, a, t, err, st, hook);
  if (e != hipSuccess) return e;
  launch_push_list<Real>(g, f, s, c, list, nlist, nlist_total, err, st);
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_push_tiled_pair(const GridInfo& g, const FieldPtrs<Real>& f,
                                  const SpeciesDev<Real>& si, const PushConst<Real>& ci,
                                  const uint32_t* tile_off_i, uint32_t* list_i,
                                  uint32_t* defer_i, const SpeciesDev<Real>& se,
                                  const PushConst<Real>& ce, const uint32_t* tile_off_e,
                                  uint32_t* list_e, const TileGeom& t, uint32_t* nlist,
                                  uint32_t* total_i, uint32_t* total_e, uint32_t* nfar_i,
                                  uint32_t* err, hipStream_t st, DispatchHook hook) {
  hipError_t e = hipMemsetAsync(nlist, 0, 2 * sizeof(uint32_t), st);
  if (e != hipSuccess) return e;
  const TileSpecies<Real> a = tile_species(si, ci, tile_off_i, list_i, nlist, nfar_i, defer_i);
  const TileSpecies<Real> b =
      tile_species(se, ce, tile_off_e, list_e, nlist + 1, nfar_i, (uint32_t*)nullptr);
  e = launch_colours<Real, 2>(g, f, a, b, t, err, st, hook);
  if (e != hipSuccess) return e;
  if (si.n > 0) launch_push_list<Real>(g, f, si, ci, list_i, nlist, total_i, err, st);
  if (se.n > 0) launch_push_list<Real>(g, f, se, ce, list_e, nlist + 1, total_e, err, st);
  return hipGetLastError();
}

template hipError_t launch_push_tiled<float>(const GridInfo&, const FieldPtrs<float>&,
                                             const SpeciesDev<float>&, const PushConst<float>&,
                                             const TileGeom&, const uint32_t*, uint32_t*,
                                             uint32_t*, uint32_t*, uint32_t*, uint32_t*,
                                             uint32_t*, hipStream_t, DispatchHook);
template hipError_t launch_push_tiled<double>(const GridInfo&, const FieldPtrs<double>&,
                                              const SpeciesDev<double>&, const PushConst<double>&,
                                              const TileGeom&, const uint32_t*, uint32_t*,
                                              uint32_t*, uint32_t*, uint32_t*, uint32_t*,
                                              uint32_t*, hipStream_t, DispatchHook);
template hipError_t launch_push_tiled_pair<float>(
    const GridInfo&, const FieldPtrs<float>&, const SpeciesDev<float>&, const PushConst<float>&,
    const uint32_t*, uint32_t*, uint32_t*, const SpeciesDev<float>&, const PushConst<float>&,
    const uint32_t*, uint32_t*, const TileGeom&, uint32_t*, uint32_t*, uint32_t*, uint32_t*,
    uint32_t*, hipStream_t, DispatchHook);
template hipError_t launch_push_tiled_pair<double>(
    const GridInfo&, const FieldPtrs<double>&, const SpeciesDev<double>&,
    const PushConst<double>&, const uint32_t*, uint32_t*, uint32_t*, const SpeciesDev<double>&,
    const PushConst<double>&, const uint32_t*, uint32_t*, const TileGeom&, uint32_t*, uint32_t*,
    uint32_t*, uint32_t*, uint32_t*, hipStream_t, DispatchHook);

}  // namespace pic
