// sort.hip -- stable LSD radix sorts of particles by tile id.
//
// Digits of up to 9 bits (a key of b bits takes ceil(b / 9) passes, the
// digit width spread evenly over them: 17-bit tile ids of a 512x256x256
// grid in 8x8x6 tiles sort in two passes of 9 bits).
// Pass structure (per digit): block histograms over chunks of 4096 keys,
// an exclusive scan of the digit-major histogram table, and a stable
// block scatter in which each wavefront ranks equal digits with ballots.
// The resulting permutation gathers every attribute array in one kernel.
#include <algorithm>

#include "sort.h"

namespace pic {

namespace {

constexpr int SB = 256;          // threads per block
constexpr int ROUNDS = 16;       // items per thread
constexpr int CHUNK = SB * ROUNDS;
constexpr int SCAN_ITEMS = 1024; // per scan block (4 per thread)
constexpr int MAXBITS = 9;       // widest digit
constexpr int MAXBINS = 1 << MAXBITS;

__global__ void k_keys(GridInfo g, int tx, int ty, int tz, int ntx, int nty, const uint32_t* cell,
                       int64_t n, uint32_t* key) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  uint32_t v = cell[p];
  uint32_t i = v & ((1u << g.bits[0]) - 1u);
  uint32_t j = g.nd > 1 ? (v >> g.bits[0]) & ((1u << g.bits[1]) - 1u) : 0u;
  uint32_t k = g.nd > 2 ? v >> (g.bits[0] + g.bits[1]) : 0u;
  key[p] = i / tx + (uint32_t)ntx * (j / ty + (uint32_t)nty * (k / tz));
}

// Key of the ordering sort after a load: tile id times the cells of a tile
// plus the cell's index within its tile (x fastest).
__global__ void k_cell_keys(GridInfo g, int tx, int ty, int tz, int ntx, int nty,
                            const uint32_t* cell, int64_t n, uint32_t* key) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  uint32_t v = cell[p];
  uint32_t i = v & ((1u << g.bits[0]) - 1u);
  uint32_t j = g.nd > 1 ? (v >> g.bits[0]) & ((1u << g.bits[1]) - 1u) : 0u;
  uint32_t k = g.nd > 2 ? v >> (g.bits[0] + g.bits[1]) : 0u;
  uint32_t tile = i / tx + (uint32_t)ntx * (j / ty + (uint32_t)nty * (k / tz));
  uint32_t local = i % tx + (uint32_t)tx * (j % ty + (uint32_t)ty * (k % tz));
  key[p] = tile * (uint32_t)(tx * ty * tz) + local;
}

// Over keys sorted by (tile, cell): the rank of element i among the equal
// keys before it (its rank within the cell, in the previous order), found
// by a doubling search back to the start of the run and a bisection, then
// the key (tile, rank) with the rank clamped to rmax.
__global__ void k_rank_keys(const uint32_t* __restrict__ ck, int64_t n, uint32_t cpt, int rbits,
                            uint32_t* __restrict__ rk) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t K = ck[i];
  int64_t hi = i, lo = -1;  // ck[hi] == K; lo < 0 or ck[lo] < K
  for (int64_t d = 1;; d <<= 1) {
    const int64_t q = i - d;
    if (q < 0) break;
    if (ck[q] != K) {
      lo = q;
      break;
    }
    hi = q;
  }
  while (hi - lo > 1) {
    const int64_t m = lo + (hi - lo) / 2;
    if (ck[m] == K)
      hi = m;
    else
      lo = m;
  }
  const uint32_t rmax = (1u << rbits) - 1u;
  const int64_t r = i - hi;
  const uint32_t rank = r < (int64_t)rmax ? (uint32_t)r : rmax;
  rk[i] = ((K / cpt) << rbits) | rank;
}

// Digit histogram of one chunk of keys.  The keys arrive nearly sorted
// (a re-sort moves few particles), so the lanes of a wavefront mostly share
// one digit: the lanes with equal digits are found by ballots over the
// digit's bits and one lane adds their count (one LDS atomic per distinct
// digit of a wavefront instead of one per key).
__global__ void __launch_bounds__(SB) k_hist(const uint32_t* key, int64_t n, int shift,
                                             int nbits, uint32_t* hist, int nb) {
  __shared__ uint32_t h[MAXBINS];
  const int bins = 1 << nbits;
  const uint32_t mask = (uint32_t)bins - 1u;
  const int lane = threadIdx.x & 63;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int d = threadIdx.x; d < bins; d += SB) h[d] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * CHUNK;
  // every load of the chunk issued before the first is used
  uint32_t kv[ROUNDS];
#pragma unroll
  for (int r = 0; r < ROUNDS; r++) {
    const int64_t i = base + (int64_t)r * SB + threadIdx.x;
    kv[r] = i < n ? key[i] : 0u;
  }
#pragma unroll
  for (int r = 0; r < ROUNDS; r++) {
    const int64_t i = base + (int64_t)r * SB + threadIdx.x;
    const bool valid = i < n;
    const uint32_t dig = valid ? (kv[r] >> shift) & mask : 0u;
    uint64_t m = __ballot(valid);
    for (int b = 0; b < nbits; b++) {
      const bool bit = (dig >> b) & 1u;
      const uint64_t bb = __ballot(valid && bit);
      m &= bit ? bb : ~bb;
    }
    // the lowest lane of each group of equal digits adds the group's count
    if (valid && (m & lt) == 0ull) atomicAdd(&h[dig], (uint32_t)__popcll(m));
  }
  __syncthreads();
  for (int d = threadIdx.x; d < bins; d += SB) hist[(int64_t)d * nb + blockIdx.x] = h[d];
}

// in-place exclusive scan of 1024-element blocks; block totals -> sums[b]
__global__ void __launch_bounds__(SB) k_scan_block(uint32_t* a, int64_t L, uint32_t* sums) {
  __shared__ uint32_t s[SB];
  int64_t base = (int64_t)blockIdx.x * SCAN_ITEMS + (int64_t)threadIdx.x * 4;
  uint32_t v[4], t = 0;
  for (int q = 0; q < 4; q++) {
    v[q] = (base + q < L) ? a[base + q] : 0u;
    t += v[q];
  }
  s[threadIdx.x] = t;
  __syncthreads();
  for (int off = 1; off < SB; off <<= 1) {
    uint32_t add = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0u;
    __syncthreads();
    s[threadIdx.x] += add;
    __syncthreads();
  }
  uint32_t run = s[threadIdx.x] - t;  // exclusive prefix of this thread
  for (int q = 0; q < 4; q++) {
    if (base + q < L) a[base + q] = run;
    run += v[q];
  }
  if (threadIdx.x == SB - 1) sums[blockIdx.x] = s[SB - 1];
}

__global__ void k_scan_add(uint32_t* a, int64_t L, const uint32_t* sums) {
  int64_t i = (int64_t)blockIdx.x * SCAN_ITEMS + threadIdx.x;
  uint32_t add = sums[blockIdx.x];
  for (int q = 0; q < 4; q++, i += SB)
    if (i < L) a[i] += add;
}

void scan_exclusive(uint32_t* a, int64_t L, uint32_t* tmp, hipStream_t st) {
  int64_t nb = (L + SCAN_ITEMS - 1) / SCAN_ITEMS;
  hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nb), SB, 0, st, a, L, tmp);
  if (nb > 1) {
    scan_exclusive(tmp, nb, tmp + nb, st);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), SB, 0, st, a, L, tmp);
  }
}

__global__ void __launch_bounds__(SB) k_scatter(const uint32_t* kin, const uint32_t* iin,
                                                uint32_t* kout, uint32_t* iout,
                                                const uint32_t* offs, int shift, int nbits,
                                                int64_t n, int nb) {
  __shared__ uint32_t run[MAXBINS];
  __shared__ uint32_t wc[SB / 64][MAXBINS];
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int bins = 1 << nbits;
  const uint32_t mask = (uint32_t)bins - 1u;
  for (int d = t; d < bins; d += SB) {
    run[d] = offs[(int64_t)d * nb + blockIdx.x];
    for (int q = 0; q < SB / 64; q++) wc[q][d] = 0;
  }
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = (int64_t)blockIdx.x * CHUNK;
  // every key (and index) of the chunk loaded before the rounds start
  uint32_t kv[ROUNDS], iv[ROUNDS];
#pragma unroll
  for (int r = 0; r < ROUNDS; r++) {
    const int64_t i = base + (int64_t)r * SB + t;
    kv[r] = i < n ? kin[i] : 0u;
    iv[r] = i < n ? (iin ? iin[i] : (uint32_t)i) : 0u;
  }
  __syncthreads();
  // Per round: the lowest lane of each group of equal digits in a wavefront
  // (its leader) posts the group's count in wc[wave][digit]; every key's
  // place is the digit's running offset, plus the counts of that digit in
  // the lower wavefronts, plus its rank in its group; then the leaders add
  // their counts to the running offsets and clear their wc entries, so a
  // round touches only the digits it holds.
#pragma unroll
  for (int r = 0; r < ROUNDS; r++) {
    int64_t i = base + (int64_t)r * SB + t;
    bool valid = i < n;
    uint32_t key = kv[r];
    uint32_t dig = (key >> shift) & mask;
    // lanes of this wavefront with the same digit, by ballots over its bits
    uint64_t m = __ballot(valid);
    for (int b = 0; b < nbits; b++) {
      bool bit = (dig >> b) & 1u;
      uint64_t bb = __ballot(valid && bit);
      m &= bit ? bb : ~bb;
    }
    const uint32_t rank = (uint32_t)__popcll(m & lt), cnt = (uint32_t)__popcll(m);
    const bool leader = valid && rank == 0;
    if (leader) wc[wave][dig] = cnt;
    __syncthreads();
    uint32_t pos = 0;
    if (valid) {
      pos = run[dig] + rank;
      for (int q = 0; q < wave; q++) pos += wc[q][dig];
    }
    __syncthreads();
    if (leader) {
      atomicAdd(&run[dig], cnt);
      wc[wave][dig] = 0;
    }
    if (valid) {
      kout[pos] = key;
      iout[pos] = iv[r];
    }
    __syncthreads();
  }
}

// Offsets of the tiles in the sorted order (the tile id is key >> tshift):
// one thread per tile boundary t in [0, ntiles], off[t] = the number of
// keys whose tile is below t, by binary search (a run of empty tiles costs
// nothing, unlike filling it from the particle side).
__global__ void k_tile_off(const uint32_t* key, int64_t n, int64_t ntiles, int tshift,
                           uint32_t* off) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t > ntiles) return;
  int64_t lo = 0, hi = n;  // first index whose tile is >= t lies in [lo, hi]
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if ((int64_t)(key[mid] >> tshift) < t)
      lo = mid + 1;
    else
      hi = mid;
  }
  off[t] = (uint32_t)lo;
}

// Every attribute of element i gathered through one read of the
// permutation: up to kMaxAttr arrays of 4- or 8-byte elements.
struct GatherSet {
  const void* src[kMaxAttr];
  void* dst[kMaxAttr];
  int wide[kMaxAttr];  // 8-byte elements
  int n;
};

__global__ void __launch_bounds__(256) k_gather_all(GatherSet gs,
                                                    const uint32_t* __restrict__ idx,
                                                    int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t j = idx[i];
  // all loads first (independent, in flight together), then the stores
  uint64_t v[kMaxAttr];
#pragma unroll
  for (int a = 0; a < kMaxAttr; a++) {
    if (a < gs.n)
      v[a] = gs.wide[a] ? static_cast<const uint64_t*>(gs.src[a])[j]
                        : (uint64_t) static_cast<const uint32_t*>(gs.src[a])[j];
  }
#pragma unroll
  for (int a = 0; a < kMaxAttr; a++) {
    if (a < gs.n) {
      if (gs.wide[a])
        static_cast<uint64_t*>(gs.dst[a])[i] = v[a];
      else
        static_cast<uint32_t*>(gs.dst[a])[i] = (uint32_t)v[a];
    }
  }
}

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

int sort_alloc(const GridInfo&, const int ntiles[3], int64_t cap, const AllocFn& alloc,
               SortBuffers& sb) {
  sb.cap = cap;
  sb.ntiles = (int64_t)ntiles[0] * ntiles[1] * ntiles[2];
  int64_t nb = (cap + CHUNK - 1) / CHUNK;
  int64_t hist = (int64_t)MAXBINS * nb;
  int64_t tmp = hist / 512 + 4096;
  for (int b = 0; b < 2; b++) {
    sb.key[b] = static_cast<uint32_t*>(alloc(cap * 4));
    sb.idx[b] = static_cast<uint32_t*>(alloc(cap * 4));
    if (!sb.key[b] || !sb.idx[b]) return -1;
  }
  sb.hist = static_cast<uint32_t*>(alloc(hist * 4));
  sb.scan_tmp = static_cast<uint32_t*>(alloc(tmp * 4));
  sb.tile_off = static_cast<uint32_t*>(alloc((sb.ntiles + 1) * 4));
  if (!sb.hist || !sb.scan_tmp || !sb.tile_off) return -1;
  // until the first sort every tile is empty
  if (hipMemset(sb.tile_off, 0, (sb.ntiles + 1) * 4) != hipSuccess) return -1;
  return 0;
}

int sort_add_attr(SortBuffers& sb, void** ptr, size_t elem, const AllocFn& alloc) {
  if (sb.nattr >= kMaxSortAttr) return -1;
  void* a = alloc(sb.cap * elem);
  if (!a) return -1;
  sb.attr[sb.nattr] = ptr;
  sb.elem[sb.nattr] = elem;
  sb.alt[sb.nattr] = a;
  sb.nattr++;
  return 0;
}

// Stable LSD radix sort of the n keys in sb.key[kc] (bits wide) carrying
// the indices in sb.idx[ic] (identity when ic < 0); kc and ic name the
// buffers that hold the result on return.
static void radix_sort(SortBuffers& sb, int64_t n, int bits, int& kc, int& ic, hipStream_t st) {
  const int passes = (bits + MAXBITS - 1) / MAXBITS;
  const int dbits = passes ? (bits + passes - 1) / passes : 0;
  const int nb = (int)((n + CHUNK - 1) / CHUNK);
  for (int p = 0; p < passes; p++) {
    const int shift = dbits * p;
    const int ko = 1 - kc, io = ic < 0 ? 0 : 1 - ic;
    hipLaunchKernelGGL(k_hist, dim3(nb), SB, 0, st, sb.key[kc], n, shift, dbits, sb.hist, nb);
    scan_exclusive(sb.hist, ((int64_t)1 << dbits) * nb, sb.scan_tmp, st);
    hipLaunchKernelGGL(k_scatter, dim3(nb), SB, 0, st, sb.key[kc], ic < 0 ? nullptr : sb.idx[ic],
                       sb.key[ko], sb.idx[io], sb.hist, shift, dbits, n, nb);
    kc = ko;
    ic = io;
  }
}

static int bits_for(uint64_t count) {
  int b = 0;
  while ((uint64_t(1) << b) < count) b++;
  return b;
}

int sort_by_tile(const GridInfo& g, const int tile[3], const int ntiles[3], SortBuffers& sb,
                 int64_t n, hipStream_t st, bool interleave) {
  if (n <= 0) return 0;
  uint32_t* cell = static_cast<uint32_t*>(*sb.attr[0]);
  const uint64_t cpt = (uint64_t)tile[0] * tile[1] * tile[2];
  const int tbits = bits_for((uint64_t)sb.ntiles);
  const int rbits = 32 - tbits < 8 ? 32 - tbits : 8;
  // the ordering sort needs (tile, cell) and (tile, rank) keys of 32 bits
  interleave = interleave && cpt > 1 && rbits > 0 &&
               (uint64_t)sb.ntiles * cpt <= (uint64_t)UINT32_MAX;
  int kc = 0, ic = -1, tshift = 0;
  if (interleave) {
    hipLaunchKernelGGL(k_cell_keys, nblk(n, 256), 256, 0, st, g, tile[0], tile[1], tile[2],
                       ntiles[0], ntiles[1], cell, n, sb.key[0]);
    radix_sort(sb, n, bits_for((uint64_t)sb.ntiles * cpt), kc, ic, st);
    hipLaunchKernelGGL(k_rank_keys, nblk(n, 256), 256, 0, st, sb.key[kc], n, (uint32_t)cpt, rbits,
                       sb.key[1 - kc]);
    kc = 1 - kc;
    radix_sort(sb, n, tbits + rbits, kc, ic, st);
    tshift = rbits;
  } else {
    hipLaunchKernelGGL(k_keys, nblk(n, 256), 256, 0, st, g, tile[0], tile[1], tile[2], ntiles[0],
                       ntiles[1], cell, n, sb.key[0]);
    radix_sort(sb, n, tbits, kc, ic, st);
  }
  hipLaunchKernelGGL(k_tile_off, nblk(sb.ntiles + 1, 256), 256, 0, st, sb.key[kc], n, sb.ntiles,
                     tshift, sb.tile_off);
  if (ic < 0) return hipGetLastError() == hipSuccess ? 0 : -1;  // a single tile: order unchanged
  const uint32_t* perm = sb.idx[ic];
  for (int a0 = 0; a0 < sb.nattr; a0 += kMaxAttr) {
    GatherSet gs{};
    gs.n = std::min(kMaxAttr, sb.nattr - a0);
    for (int a = 0; a < gs.n; a++) {
      gs.src[a] = *sb.attr[a0 + a];
      gs.dst[a] = sb.alt[a0 + a];
      gs.wide[a] = sb.elem[a0 + a] == 8;
    }
    hipLaunchKernelGGL(k_gather_all, nblk(n, 256), 256, 0, st, gs, perm, n);
  }
  for (int a = 0; a < sb.nattr; a++) {
    void* src = *sb.attr[a];
    *sb.attr[a] = sb.alt[a];
    sb.alt[a] = src;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace pic
