// k_build.hip -- level-order octree and i-groups from sorted Morton keys.
//
// Tree definition (the paper's makeTree, Sec. 2.2; details it leaves open):
// a cell at level l holds the particles whose key >> 3(21-l) equals its
// prefix; it is split iff it holds more than leaf_max particles and l < 21;
// only non-empty octants become children, consecutive in octant order; cells
// are numbered by level, then by prefix.
//
// Construction without a per-level host loop. For sorted keys K and
// cpl(a, b) = number of leading octant digits K[a] and K[b] share:
//  * particle i starts a run of equal level-l prefix iff l > cpl(i-1, i);
//    let s_i = cpl(i-1, i) + 1 (s_0 = 0);
//  * the level-l cell of i holds more than W particles iff some window of
//    W+1 consecutive particles containing i shares its level-l prefix, i.e.
//    iff l <= M_i(W) = max over s in [i-W, i] of cpl(s, s+W);
//  * cells containing i exist at levels 0..D_i with D_i = min(M_i(leaf_max)
//    + 1, 21).
// So particle i starts the cells (l, i) for s_i <= l <= D_i, and its leaf iff
// s_i <= D_i; its cells at levels up to E_i = M_i(64) hold more than 64
// particles (calcNode treats those and the smaller ones differently). The level-order
// index of (l, i) is the number of cells of lower level plus the number of
// level-l cells starting before i: per-level block counts, a scan over
// blocks, and ballots inside the block give it. The window maxima use a
// sparse table (doubling) in LDS.
//
// i-groups (the particles sharing one interaction list, Sec. 1) are the cells
// holding at most group_max particles whose parent holds more (the root if
// it holds at most group_max); an oversized level-21 cell is cut into pieces
// of group_max. With group_merge, consecutive sibling group cells are joined
// greedily in octant order while the joined count stays within group_max
// (siblings within one system only: a batch's system roots are never joined).
// Each cell holding more than group_max particles marks the group starts
// among its children; a scan over the marked particles lists the groups in
// particle order.
#include <algorithm>

#include "nbody_internal.h"

namespace nb {

constexpr int kB = kBuildThreads;
constexpr int kH = kBuildHalo;
constexpr uint32_t kGroupMark = 1u << 15;  // pinfo: particle starts a group

__device__ __forceinline__ int cpl_keys(uint64_t a, uint64_t b) {
  const uint64_t x = a ^ b;
  if (x == 0) return kMaxLevel;
  return (__clzll(x) - 1) / 3;
}

// In-place doubling: t[s] <- max(t[s .. s + 2^k - 1]) for the valid prefix.
__device__ void lds_window_max(int *t, int len, int k) {
  for (int j = 0; j < k; ++j) {
    const int d = 1 << j;
    int a0 = -1, a1 = -1;
    const int t0 = threadIdx.x, t1 = threadIdx.x + kB;
    if (t0 < len) a0 = max(t[t0], t0 + d < len ? t[t0 + d] : -1);
    if (t1 < len) a1 = max(t[t1], t1 + d < len ? t[t1 + d] : -1);
    __syncthreads();
    if (t0 < len) t[t0] = a0;
    if (t1 < len) t[t1] = a1;
    __syncthreads();
  }
}

__device__ __forceinline__ int ilog2_floor(int v) { return 31 - __clz(v); }

// Pass A: per sorted particle s_i, D_i and E_i; per block and level the
// number of cells starting in the block, and (row kLevels) of leaves.
constexpr int kBigCell = 64;  // cells holding more particles are "big" (E_i)
static_assert(kH >= kBigCell, "the halo covers the window of a big cell");

__global__ __launch_bounds__(kB) void k_build_a(const uint64_t *__restrict__ K,
                                                uint32_t n, int leaf_max, int min_level,
                                                uint32_t *__restrict__ pinfo,
                                                uint32_t *__restrict__ blkcnt,
                                                uint32_t nblk) {
  __shared__ uint64_t sk[kB + 2 * kH];
  __shared__ int tL[kB + kH];
  __shared__ int tE[kB + kH];
  __shared__ uint32_t wc[kLevels + 1][kB / 64];
  const int64_t b0 = (int64_t)blockIdx.x * kB;
  for (int t = threadIdx.x; t < kB + 2 * kH; t += kB) {
    const int64_t pos = b0 - kH + t;
    sk[t] = (pos >= 0 && pos < n) ? K[pos] : 0ull;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < kB + kH; t += kB) {
    const int64_t s = b0 - kH + t;
    tL[t] = (s >= 0 && s + leaf_max < n) ? cpl_keys(sk[t], sk[t + leaf_max]) : -1;
    tE[t] = (s >= 0 && s + kBigCell < n) ? cpl_keys(sk[t], sk[t + kBigCell]) : -1;
  }
  __syncthreads();
  const int kLw = ilog2_floor(leaf_max + 1);
  lds_window_max(tL, kB + kH, kLw);
  constexpr int kEw = 6;  // floor(log2(kBigCell + 1))
  lds_window_max(tE, kB + kH, kEw);
  const int64_t i = b0 + threadIdx.x;
  const bool valid = i < n;
  const int li = threadIdx.x + kH;
  int s = 0, D = 0;
  if (valid) {
    s = (i == 0) ? 0 : cpl_keys(sk[li - 1], sk[li]) + 1;
    const int M = max(tL[li - leaf_max], tL[li - (1 << kLw) + 1]);
    D = max(min(M + 1, kMaxLevel), min_level);  // cells above min_level always split
    const int E = max(tE[li - kBigCell], tE[li - (1 << kEw) + 1]);  // -1: no big cell
    // group mark (bit 15) clear
    pinfo[i] = (uint32_t)s | ((uint32_t)D << 5) | ((uint32_t)(E + 1) << 10);
  }
  const int w = threadIdx.x >> 6;
  for (int l = 0; l < kLevels; ++l) {
    const uint64_t b = __ballot(valid && s <= l && l <= D);
    if (lane_id() == 0) wc[l][w] = (uint32_t)__popcll(b);
  }
  {
    const uint64_t b = __ballot(valid && s <= D);  // leaf starts
    if (lane_id() == 0) wc[kLevels][w] = (uint32_t)__popcll(b);
  }
  __syncthreads();
  if (threadIdx.x <= kLevels) {
    uint32_t t = 0;
    for (int q = 0; q < kB / 64; ++q) t += wc[threadIdx.x][q];
    blkcnt[threadIdx.x * nblk + blockIdx.x] = t;
  }
}

// Exclusive scan of each row of rows[row][0 .. len) in place, the row total
// to totals[row], in three coalesced passes over tiles of kScanTile entries:
// tile sums, a scan of each row's tile sums (into tsum), then every tile
// rescanned with its offset.
constexpr uint32_t kScanTile = 4096;  // 256 threads x 16

__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t v, uint32_t *wsum,
                                                       uint32_t *total) {
  const uint32_t inc = wave_incl_scan_dpp(v);
  const int w = threadIdx.x >> 6;
  if (lane_id() == 63) wsum[w] = inc;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    off += q < w ? wsum[q] : 0u;
    tot += wsum[q];
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

__global__ __launch_bounds__(256) void k_scan_tiles(const uint32_t *__restrict__ rows,
                                                    uint32_t len, uint32_t ntile,
                                                    uint32_t *__restrict__ tsum) {
  __shared__ uint32_t wsum[4];
  const uint32_t *row = rows + (size_t)blockIdx.y * len;
  const uint32_t b = blockIdx.x * kScanTile;
  uint32_t s = 0;
#pragma unroll
  for (uint32_t k = 0; k < kScanTile / 256; ++k) {
    const uint32_t j = b + k * 256u + threadIdx.x;
    s += j < len ? row[j] : 0u;
  }
  uint32_t tot;
  (void)block_excl_scan256(s, wsum, &tot);
  if (threadIdx.x == 0) tsum[(size_t)blockIdx.y * ntile + blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_scan_tilesums(uint32_t *__restrict__ tsum,
                                                       uint32_t ntile,
                                                       uint32_t *__restrict__ totals) {
  __shared__ uint32_t wsum[4];
  uint32_t *t = tsum + (size_t)blockIdx.x * ntile;
  uint32_t carry = 0;
  for (uint32_t k0 = 0; k0 < ntile; k0 += 256) {
    const uint32_t k = k0 + threadIdx.x;
    const uint32_t v = k < ntile ? t[k] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan256(v, wsum, &tot);
    if (k < ntile) t[k] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

__global__ __launch_bounds__(256) void k_scan_apply(uint32_t *__restrict__ rows, uint32_t len,
                                                    uint32_t ntile,
                                                    const uint32_t *__restrict__ tsum) {
  __shared__ uint32_t wsum[4];
  uint32_t *row = rows + (size_t)blockIdx.y * len;
  const uint32_t b = blockIdx.x * kScanTile + threadIdx.x * (kScanTile / 256);
  uint32_t v[kScanTile / 256];
  uint32_t s = 0;
#pragma unroll
  for (uint32_t k = 0; k < kScanTile / 256; ++k) {
    v[k] = b + k < len ? row[b + k] : 0u;
    s += v[k];
  }
  uint32_t tot;
  uint32_t run = tsum[(size_t)blockIdx.y * ntile + blockIdx.x] + block_excl_scan256(s, wsum, &tot);
#pragma unroll
  for (uint32_t k = 0; k < kScanTile / 256; ++k) {
    if (b + k < len) row[b + k] = run;
    run += v[k];
  }
}

void launch_scan_rows(uint32_t *rows, uint32_t len, int nrows, uint32_t *totals,
                      uint32_t *tsum, hipStream_t st) {
  const uint32_t ntile = (uint32_t)std::max<int64_t>(cdiv(len, kScanTile), 1);
  hipLaunchKernelGGL(k_scan_tiles, dim3(ntile, nrows), dim3(256), 0, st, rows, len, ntile, tsum);
  hipLaunchKernelGGL(k_scan_tilesums, dim3(nrows), dim3(256), 0, st, tsum, ntile, totals);
  hipLaunchKernelGGL(k_scan_apply, dim3(ntile, nrows), dim3(256), 0, st, rows, len, ntile, tsum);
}

int64_t scan_scratch_words(int64_t len, int nrows) {
  return std::max<int64_t>(cdiv(len, kScanTile), 1) * nrows;
}

// Pass C: level offsets and the cell count.
__global__ void k_build_c(const uint32_t *__restrict__ totals, DevScalars *sc,
                          int64_t cell_cap) {
  if (threadIdx.x != 0) return;
  sc->nleaf = totals[kLevels];
  uint32_t o = 0;
  for (int l = 0; l < kLevels; ++l) {
    sc->lvl_off[l] = o;
    o += totals[l];
  }
  sc->lvl_off[kLevels] = o;
  if ((int64_t)o > cell_cap) {
    atomicOr(&sc->status, kStCapacity);
    o = 0;
  }
  sc->ncell = o;
}

// Pass D: write every cell (l, i). The level-l run from i (the cell's
// particles) ends at the first j > i with s_j <= l, where s_j - 1 is the
// number of leading octant digits K[j-1] and K[j] share: K[j] leaves i's
// level-l prefix exactly there. So for the 512 positions from the block's
// start the pass keeps, per level L, bit masks of {j : s_j <= L} (64-bit
// ballots); a run end is the first set bit after i and a child count the
// number of set bits inside the run (level l + 1). The cells starting in a
// wavefront's 64 particles are dealt out to its lanes, one cell per lane and
// round. A run longer than kShort goes to a queue that k_build_long serves
// with a whole wavefront per cell (64 probes per round).
constexpr uint32_t kShort = kB;
constexpr uint32_t kLongCell = 0xffffffffu;   // cpcount of a cell left to k_build_long
constexpr int kSpan = 2 * kB;                 // positions with masks: [b0, b0 + 2 kB)
constexpr int kChunks = kSpan / 64;
constexpr int kTasksPerWave = 64 * kLevels;   // (lane, level) pairs of one wavefront

// First set bit of masks m[0 .. kChunks) at relative positions (r0, r1]; -1 if none.
__device__ __forceinline__ int first_bit(const uint64_t *m, uint32_t r0, uint32_t r1) {
  for (uint32_t c = (r0 + 1) >> 6; c <= (r1 >> 6); ++c) {
    uint64_t v = m[c];
    if (c == ((r0 + 1) >> 6)) v &= ~0ull << ((r0 + 1) & 63);
    if (c == (r1 >> 6) && (r1 & 63) != 63) v &= (2ull << (r1 & 63)) - 1;
    if (v) return (int)(c * 64 + __builtin_ctzll(v));
  }
  return -1;
}

// Number of set bits of m at relative positions (r0, r1).
__device__ __forceinline__ uint32_t count_bits(const uint64_t *m, uint32_t r0, uint32_t r1) {
  if (r1 <= r0 + 1) return 0;
  const uint32_t lo = r0 + 1, hi = r1 - 1;  // inclusive
  uint32_t t = 0;
  for (uint32_t c = lo >> 6; c <= (hi >> 6); ++c) {
    uint64_t v = m[c];
    if (c == (lo >> 6)) v &= ~0ull << (lo & 63);
    if (c == (hi >> 6) && (hi & 63) != 63) v &= (2ull << (hi & 63)) - 1;
    t += (uint32_t)__popcll(v);
  }
  return t;
}

__global__ __launch_bounds__(kB) void k_build_d(
    const uint32_t *__restrict__ pinfo, uint32_t n, const uint32_t *__restrict__ blkcnt,
    uint32_t nblk, DevScalars *__restrict__ sc, int64_t cell_cap,
    int32_t *__restrict__ clevel, uint32_t *__restrict__ cpbegin,
    uint32_t *__restrict__ cpcount, int32_t *__restrict__ cfchild,
    int32_t *__restrict__ cnchild, float4 *__restrict__ nodeB,
    uint32_t *__restrict__ leafof, uint2 *__restrict__ leaves,
    uint32_t *__restrict__ longcnt, uint32_t *__restrict__ longslot) {
  __shared__ uint32_t s_nlong;  // cells longer than kShort starting in this block
  __shared__ uint32_t wpre[kLevels + 1][kB / 64];  // row kLevels: leaf starts
  __shared__ uint32_t lvl_off[kLevels + 1];
  __shared__ uint64_t bound[kLevels][kChunks];       // bit j: s_{b0+j} <= level (or past n)
  __shared__ uint64_t wbal[kB / 64][kLevels];        // per wave and level: lanes starting a cell
  __shared__ uint8_t s_lo[kB];                       // per particle: first level it starts
  __shared__ uint16_t tasks[kB / 64][kTasksPerWave];  // (lane << 5) | level
  const uint32_t b0 = blockIdx.x * kB;
  const int64_t i = (int64_t)b0 + threadIdx.x;
  const bool valid = i < n;
  const int w = threadIdx.x >> 6;
  const uint32_t lane = lane_id();
  if (threadIdx.x == 0) s_nlong = 0;
  // boundary masks: wave w covers chunks 2w and 2w + 1
  for (int c = 2 * w; c < 2 * w + 2; ++c) {
    const int64_t q = (int64_t)b0 + c * 64 + lane;
    const int sq = q < n ? (int)(pinfo[q] & 31u) : 0;
    for (int L = 0; L < kLevels; ++L) {
      const uint64_t m = __ballot(sq <= L);
      if (lane == 0) bound[L][c] = m;
    }
  }
  const uint32_t pi = valid ? pinfo[i] : 0u;
  const int s = pi & 31, D = (pi >> 5) & 31;
  if (threadIdx.x <= kLevels) lvl_off[threadIdx.x] = sc->lvl_off[threadIdx.x];
  for (int l = 0; l < kLevels; ++l) {
    const uint64_t b = __ballot(valid && s <= l && l <= D);
    if (lane == 0) {
      wpre[l][w] = (uint32_t)__popcll(b);
      wbal[w][l] = b;
    }
  }
  const uint64_t lbal = __ballot(valid && s <= D);  // this wave's leaf starts
  if (lane == 0) wpre[kLevels][w] = (uint32_t)__popcll(lbal);
  s_lo[threadIdx.x] = (uint8_t)s;
  // this lane's cells as tasks of its wave, in lane order
  const uint32_t nt = (valid && s <= D) ? (uint32_t)(D - s + 1) : 0u;
  const uint32_t tinc = wave_incl_scan(nt);
  const uint32_t ntask = __builtin_amdgcn_readlane(tinc, 63);
  for (uint32_t t = 0; t < nt; ++t) tasks[w][tinc - nt + t] = (uint16_t)((lane << 5) | (s + t));
  __syncthreads();
  if (threadIdx.x <= kLevels) {
    uint32_t o = 0;
    for (int q = 0; q < kB / 64; ++q) {
      const uint32_t t = wpre[threadIdx.x][q];
      wpre[threadIdx.x][q] = o;
      o += t;
    }
  }
  __syncthreads();
  // the leaf list, in particle order: (leaf cell, first particle); the
  // particle's leaf is its cell at level D
  if (valid && s <= D) {
    const uint32_t rank = blkcnt[(int64_t)kLevels * nblk + blockIdx.x] + wpre[kLevels][w] +
                          (uint32_t)__popcll(lbal & lanemask_lt());
    const uint32_t lrank = blkcnt[(int64_t)D * nblk + blockIdx.x] + wpre[D][w] +
                           (uint32_t)__popcll(wbal[w][D] & lanemask_lt());
    leaves[rank] = make_uint2(lvl_off[D] + lrank, (uint32_t)i);
  }
  for (uint32_t t = lane; t < ntask; t += 64) {
    const uint32_t code = tasks[w][t];
    const uint32_t k = code >> 5;  // the lane (particle) starting the cell
    const int l = (int)(code & 31u);
    const uint32_t r = (uint32_t)w * 64u + k;  // position relative to b0
    const uint32_t ip = b0 + r;
    const uint64_t below = (k == 0) ? 0ull : (~0ull >> (64 - k));
    const uint32_t rank = blkcnt[(int64_t)l * nblk + blockIdx.x] + wpre[l][w] +
                          (uint32_t)__popcll(wbal[w][l] & below);
    const uint32_t idx = lvl_off[l] + rank;
    if ((int64_t)idx >= cell_cap) continue;
    if (l > (int)s_lo[r]) {  // (l-1, ip) is internal: this is its first child
      const uint32_t rp = blkcnt[(int64_t)(l - 1) * nblk + blockIdx.x] + wpre[l - 1][w] +
                          (uint32_t)__popcll(wbal[w][l - 1] & below);
      const uint32_t pidx = lvl_off[l - 1] + rp;
      if ((int64_t)pidx < cell_cap) cfchild[pidx] = (int32_t)idx;
    }
    clevel[idx] = l;
    cpbegin[idx] = ip;
    const int e = first_bit(bound[l], r, r + kShort);
    if (e < 0) {  // longer than kShort: counted by the cooperative pass
      cpcount[idx] = kLongCell;
      // at most one such cell per level starts in a block of kShort
      // particles (an earlier one of its level would end inside the block)
      const uint32_t slot = atomicAdd(&s_nlong, 1u);
      if (slot < (uint32_t)kLevels) longslot[(size_t)blockIdx.x * kLevels + slot] = idx;
      else atomicOr(&sc->status, kStCorrupt);
      continue;
    }
    const uint32_t end = b0 + (uint32_t)e;
    const uint32_t cnt = end - ip;
    cpcount[idx] = cnt;
    uint32_t *wB = reinterpret_cast<uint32_t *>(&nodeB[idx]);
    if (l == (int)((pinfo[ip] >> 5) & 31u)) {  // leaf
      cfchild[idx] = -1;
      cnchild[idx] = 0;
      wB[2] = ip;
      wB[3] = cnt | kLeafBit;
      for (uint32_t p = ip; p < end; ++p) leafof[p] = idx;
    } else {
      // children: the level-(l+1) runs inside [ip, end)
      const int nc = 1 + (int)count_bits(bound[l + 1], r, (uint32_t)e);
      cnchild[idx] = nc;
      wB[3] = (uint32_t)nc;
      // wB[2] (first child) is written by pass E
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) longcnt[blockIdx.x] = min(s_nlong, (uint32_t)kLevels);
}

// End of the level-l run from i, searched by the whole wavefront: a round of
// 32 exponential probes, then rounds of 63 evenly spaced probes, each
// narrowing the bracket (K[lo] in the run, position hi past it) 64-fold.
// Every lane returns the same value; all lanes must call it together.
__device__ uint32_t wave_run_end(const uint64_t *__restrict__ K, uint32_t n, uint32_t i, int l) {
  if (l == 0) return n;
  const int sh = 3 * (kMaxLevel - l);
  const uint64_t p = K[i] >> sh;
  const uint32_t lane = lane_id();
  uint32_t lo = i, hi;
  {
    const uint64_t q = (uint64_t)i + (1ull << (lane & 31));
    const bool past = lane < 32 && (q >= n || (K[q] >> sh) != p);
    const uint64_t m = __ballot(past);  // lane 31 probes i + 2^31 >= n: never empty
    const uint32_t t = (uint32_t)__builtin_ctzll(m);
    const uint64_t e = (uint64_t)i + (1ull << t);
    hi = e < n ? (uint32_t)e : n;
    lo = t == 0 ? i : i + (1u << (t - 1));
  }
  while (hi - lo > 1) {
    const uint32_t step = (hi - lo + 63) / 64;
    const uint64_t q = (uint64_t)lo + (uint64_t)(lane + 1) * step;
    const bool in = lane < 63 && q < hi;
    const bool past = in && (K[q] >> sh) != p;
    const uint64_t m = __ballot(past);
    const uint64_t mi = __ballot(in);
    if (m == 0) {
      lo = lo + (uint32_t)(64 - __builtin_clzll(mi)) * step;  // the last probe in range
    } else {
      const uint32_t t = (uint32_t)__builtin_ctzll(m);
      hi = lo + (t + 1) * step;
      lo = lo + t * step;
    }
  }
  return hi;
}

// The cells pass D left (count still kLongCell), listed per build block:
// wavefront w takes blocks w, w + nw, ... (nw wavefronts; the long cells sit
// together in the dense regions, so dealing blocks out one at a time spreads
// them) and serves their cells one after the other, finding the cell's end
// and, for an internal cell, its number of children.
__global__ __launch_bounds__(256) void k_build_long(
    const uint64_t *__restrict__ K, uint32_t n, const uint32_t *__restrict__ pinfo,
    const DevScalars *__restrict__ sc, const int32_t *__restrict__ clevel,
    const uint32_t *__restrict__ cpbegin, uint32_t *__restrict__ cpcount,
    int32_t *__restrict__ cfchild, int32_t *__restrict__ cnchild,
    float4 *__restrict__ nodeB, uint32_t *__restrict__ leafof,
    const uint32_t *__restrict__ longcnt, const uint32_t *__restrict__ longslot,
    uint32_t nblk) {
  const uint32_t nc = sc->ncell;
  const uint32_t lane = lane_id();
  const uint32_t nw = gridDim.x * (blockDim.x >> 6);
  const uint32_t wv = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) +
                                                     (threadIdx.x >> 6));
  for (uint32_t bk = wv; bk < nblk; bk += nw) {
    const uint32_t cntb = __builtin_amdgcn_readfirstlane(longcnt[bk]);
    for (uint32_t q = 0; q < cntb; ++q) {
      const uint32_t idx =
          __builtin_amdgcn_readfirstlane(longslot[(size_t)bk * kLevels + q]);
      if (idx >= nc) continue;
      const int l = clevel[idx];
      const uint32_t i = cpbegin[idx];
      const int D = (pinfo[i] >> 5) & 31;
      const uint32_t end = wave_run_end(K, n, i, l);
      const uint32_t cnt = end - i;
      uint32_t *wB = reinterpret_cast<uint32_t *>(&nodeB[idx]);
      if (l == D) {  // leaf (an oversized level-21 cell)
        if (lane == 0) {
          cfchild[idx] = -1;
          cnchild[idx] = 0;
          wB[2] = i;
          wB[3] = cnt | kLeafBit;
        }
        for (uint32_t p = i + lane; p < end; p += 64) leafof[p] = idx;
      } else {
        // the children: the level-(l+1) cells from the first child (pass D
        // wrote it) that begin before end (cells of a level are numbered in
        // particle order, so they follow one another)
        const uint32_t f = (uint32_t)cfchild[idx];
        const uint32_t lend = sc->lvl_off[l + 2 <= kLevels ? l + 2 : kLevels];
        const uint32_t c1 = f + 1u + lane;
        const bool more = lane < 7u && c1 < lend && cpbegin[c1] < end;
        const int nch = 1 + (int)__popcll(__ballot(more));
        if (lane == 0) {
          cnchild[idx] = nch;
          wB[3] = (uint32_t)nch;
        }
      }
      if (lane == 0) cpcount[idx] = cnt;
    }
  }
}

// Pass E: parents and the first-child word of internal walk nodes.
__global__ __launch_bounds__(256) void k_build_e(DevScalars *__restrict__ sc,
                                                 const int32_t *__restrict__ clevel,
                                                 const int32_t *__restrict__ cfchild,
                                                 const int32_t *__restrict__ cnchild,
                                                 int32_t *__restrict__ cparent,
                                                 float4 *__restrict__ nodeB) {
  const uint32_t nc = sc->ncell;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nc; c += stride) {
    if (c == 0) cparent[0] = -1;
    const int k = cnchild[c];
    if (k > 0) {
      const int32_t f = cfchild[c];
      const int32_t l = clevel[c];
      if (f <= (int32_t)c || k > 8 || (uint32_t)(f + k) > nc || l < 0 || l >= kMaxLevel) {
        atomicOr(&sc->status, kStCorrupt);
        continue;
      }
      reinterpret_cast<uint32_t *>(&nodeB[c])[2] = (uint32_t)f;
      for (int q = 0; q < k; ++q) cparent[f + q] = (int32_t)c;
    }
  }
}

// The list of internal cells in cell order (so level by level), entries
// (cell, first child, children, particles): internal cells per block of 256
// cells, a scan of the block counts, then each cell's rank. istart[l] is the
// rank of cell lvl_off[l] (the internal cells before level l).
__global__ __launch_bounds__(256) void k_ilist_count(const DevScalars *__restrict__ sc,
                                                     const int32_t *__restrict__ cnchild,
                                                     uint32_t *__restrict__ cblk) {
  __shared__ uint32_t wc[4];
  const uint32_t c = blockIdx.x * 256u + threadIdx.x;
  const bool in = c < sc->ncell && cnchild[c] > 0;
  const uint64_t b = __ballot(in);
  if (lane_id() == 0) wc[threadIdx.x >> 6] = (uint32_t)__popcll(b);
  __syncthreads();
  if (threadIdx.x == 0) cblk[blockIdx.x] = wc[0] + wc[1] + wc[2] + wc[3];
}

__global__ __launch_bounds__(256) void k_ilist_emit(DevScalars *__restrict__ sc,
                                                    const uint32_t *__restrict__ cpcount,
                                                    const int32_t *__restrict__ cfchild,
                                                    const int32_t *__restrict__ cnchild,
                                                    const uint32_t *__restrict__ cblk,
                                                    uint4 *__restrict__ ilist) {
  __shared__ uint32_t wc[4];
  const uint32_t nc = sc->ncell;
  const uint32_t c = blockIdx.x * 256u + threadIdx.x;
  const int k = c < nc ? cnchild[c] : 0;
  const bool in = k > 0;
  const uint64_t b = __ballot(in);
  const int w = threadIdx.x >> 6;
  if (lane_id() == 0) wc[w] = (uint32_t)__popcll(b);
  __syncthreads();
  uint32_t rank = cblk[blockIdx.x];
  for (int q = 0; q < w; ++q) rank += wc[q];
  rank += (uint32_t)__popcll(b & lanemask_lt());  // internal cells before c
  if (in) ilist[rank] = make_uint4(c, (uint32_t)cfchild[c], (uint32_t)k, cpcount[c]);
  if (c < nc)
    for (int l = 0; l < kLevels; ++l)
      if (sc->lvl_off[l] == c) sc->istart[l] = rank;
}

// Levels starting at or past the last cell (empty) and the total.
__global__ void k_ilist_total(const uint32_t *__restrict__ total, DevScalars *sc) {
  if (threadIdx.x != 0) return;
  const uint32_t t = total[0], nc = sc->ncell;
  for (int l = 0; l < kLevels; ++l)
    if (sc->lvl_off[l] >= nc) sc->istart[l] = t;
  sc->istart[kLevels] = t;
}

__device__ __forceinline__ void mark_chunks(uint32_t *__restrict__ pinfo, uint32_t b,
                                            uint32_t cnt, uint32_t gmax) {
  for (uint32_t s = 0; s < cnt; s += gmax) pinfo[b + s] |= kGroupMark;
}

// A cell may hold a group iff it is at min_level (the system digits of a
// batch) or deeper and holds at most group_max particles or is a leaf.
__device__ __forceinline__ bool group_ok(int32_t level, uint32_t cnt, int nchild,
                                         uint32_t gmax, int min_level) {
  return level >= min_level && (cnt <= gmax || nchild == 0);
}

// Group starts: the root if it may hold a group; otherwise every cell that
// may not marks the group starts among its children (joining consecutive
// small siblings when `merge` and the cell lies within one system: above
// min_level its children are the roots of distinct systems; an over-full
// leaf is cut into pieces of group_max). Every particle is marked at most
// once.
__global__ __launch_bounds__(256) void k_group_mark(DevScalars *__restrict__ sc,
                                                    const int32_t *__restrict__ clevel,
                                                    const uint32_t *__restrict__ cpbegin,
                                                    const uint32_t *__restrict__ cpcount,
                                                    const int32_t *__restrict__ cfchild,
                                                    const int32_t *__restrict__ cnchild,
                                                    uint32_t gmax, int merge, int min_level,
                                                    uint32_t *__restrict__ pinfo) {
  const uint32_t nc = sc->ncell;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nc;
       c += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t cnt = cpcount[c];
    const int k = cnchild[c];
    const bool ok = group_ok(clevel[c], cnt, k, gmax, min_level);
    if (c == 0 && ok) {
      mark_chunks(pinfo, cpbegin[0], cnt, gmax);
      continue;
    }
    if (ok || k == 0) continue;
    const int32_t f = cfchild[c];
    uint32_t run = 0;  // particles in the open joined group (0: none open)
    const bool join = merge && clevel[c] >= min_level;
    for (int q = 0; q < k; ++q) {
      const uint32_t cb = cpbegin[f + q], cc = cpcount[f + q];
      const bool cok = group_ok(clevel[f + q], cc, cnchild[f + q], gmax, min_level);
      if (cok && cc <= gmax) {
        if (join && run > 0 && run + cc <= gmax) {
          run += cc;
        } else {
          pinfo[cb] |= kGroupMark;
          run = cc;
        }
      } else {
        run = 0;
        if (cok) mark_chunks(pinfo, cb, cc, gmax);  // an over-full (level-21) leaf
      }
    }
  }
}

// Group marks per block of kB particles.
__global__ __launch_bounds__(kB) void k_group_count(uint32_t n,
                                                    const uint32_t *__restrict__ pinfo,
                                                    uint32_t *__restrict__ gblk) {
  __shared__ uint32_t wc[kB / 64];
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  const bool mk = i < n && (pinfo[i] & kGroupMark);
  const uint64_t b = __ballot(mk);
  if (lane_id() == 0) wc[threadIdx.x >> 6] = (uint32_t)__popcll(b);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int q = 0; q < kB / 64; ++q) t += wc[q];
    gblk[blockIdx.x] = t;
  }
}

// Group begins in particle order (gblk holds exclusive block offsets), and
// each particle's group (the number of group starts up to it, minus one).
__global__ __launch_bounds__(kB) void k_group_emit(uint32_t n,
                                                   const uint32_t *__restrict__ pinfo,
                                                   const uint32_t *__restrict__ gblk,
                                                   uint32_t *__restrict__ gbegin,
                                                   uint32_t *__restrict__ gid) {
  __shared__ uint32_t wc[kB / 64];
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  const bool mk = i < n && (pinfo[i] & kGroupMark);
  const uint64_t b = __ballot(mk);
  const int w = threadIdx.x >> 6;
  if (lane_id() == 0) wc[w] = (uint32_t)__popcll(b);
  __syncthreads();
  uint32_t off = gblk[blockIdx.x];
  for (int q = 0; q < w; ++q) off += wc[q];
  const uint32_t before = (uint32_t)__popcll(b & lanemask_lt());
  if (mk) gbegin[off + before] = (uint32_t)i;
  if (i < n) gid[i] = off + before + (mk ? 1u : 0u) - 1u;  // particle 0 starts group 0
}

__global__ void k_group_total(const uint32_t *__restrict__ total, uint32_t n,
                              DevScalars *sc, uint32_t *__restrict__ gbegin) {
  if (threadIdx.x != 0) return;
  sc->ngroup = total[0];
  gbegin[total[0]] = n;
}

__global__ __launch_bounds__(256) void k_group_size(const DevScalars *__restrict__ sc,
                                                    const uint32_t *__restrict__ gbegin,
                                                    uint32_t *__restrict__ gcount) {
  const uint32_t ng = sc->ngroup;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < ng;
       g += (int64_t)gridDim.x * blockDim.x)
    gcount[g] = gbegin[g + 1] - gbegin[g];
}

// Batch: each group's walk starts at its system's root, the level-r cell of
// the system (one per system, numbered by system index). Sorted positions of
// system s are [off[s], off[s+1]) as in caller order.
__global__ __launch_bounds__(256) void k_group_root(const DevScalars *__restrict__ sc,
                                                    const uint32_t *__restrict__ gbegin,
                                                    const uint32_t *__restrict__ off, int nsys,
                                                    int r, uint32_t *__restrict__ groot) {
  const uint32_t ng = sc->ngroup;
  const uint32_t base = sc->lvl_off[r];
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < ng;
       g += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t b = gbegin[g];
    int lo = 0, hi = nsys;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (off[mid] <= b)
        lo = mid;
      else
        hi = mid;
    }
    groot[g] = base + (uint32_t)lo;
  }
}

void launch_build(const uint64_t *keys, int64_t n, int leaf_max, int group_max,
                  int group_merge, int nsys, int r, const Ptrs &P, const Layout &L,
                  hipStream_t st) {
  const uint32_t nblk = (uint32_t)cdiv(n, kB);
  // block rows [kLevels][nblk], then kLevels totals; the scanned rows stay
  // for the tree's life (calcNode derives ancestor indices from them)
  // (row kLevels: leaf starts)
  uint32_t *totals = P.lvlblk + (int64_t)(kLevels + 1) * nblk;
  hipLaunchKernelGGL(k_build_a, dim3(nblk), dim3(kB), 0, st, keys, (uint32_t)n, leaf_max, r,
                     P.pinfo, P.lvlblk, nblk);
  launch_scan_rows(P.lvlblk, nblk, kLevels + 1, totals, P.scan, st);
  hipLaunchKernelGGL(k_build_c, dim3(1), dim3(64), 0, st, totals, P.sc, L.cell_cap);
  hipLaunchKernelGGL(k_build_d, dim3(nblk), dim3(kB), 0, st, P.pinfo, (uint32_t)n, P.lvlblk,
                     nblk, P.sc, L.cell_cap, P.clevel, P.cpbegin, P.cpcount, P.cfchild,
                     P.cnchild, P.nodeB, P.leafof, P.leaves, P.longcnt, P.longslot);
  hipLaunchKernelGGL(k_build_long, dim3(1024), dim3(256), 0, st, keys, (uint32_t)n, P.pinfo,
                     P.sc, P.clevel, P.cpbegin, P.cpcount, P.cfchild, P.cnchild, P.nodeB,
                     P.leafof, P.longcnt, P.longslot, nblk);
  int64_t ge = cdiv(n, 256);
  if (ge > 4096) ge = 4096;
  hipLaunchKernelGGL(k_build_e, dim3(ge), dim3(256), 0, st, P.sc, P.clevel, P.cfchild,
                     P.cnchild, P.cparent, P.nodeB);
  // internal-cell list (block counts in the group scratch, before the groups use it)
  const uint32_t cblk = (uint32_t)cdiv(L.cell_cap, 256);
  uint32_t *ib = P.blkcnt, *itot = P.blkcnt + cblk;
  hipLaunchKernelGGL(k_ilist_count, dim3(cblk), dim3(256), 0, st, P.sc, P.cnchild, ib);
  launch_scan_rows(ib, cblk, 1, itot, P.scan, st);
  hipLaunchKernelGGL(k_ilist_emit, dim3(cblk), dim3(256), 0, st, P.sc, P.cpcount, P.cfchild,
                     P.cnchild, ib, P.ilist);
  hipLaunchKernelGGL(k_ilist_total, dim3(1), dim3(64), 0, st, itot, P.sc);
  // groups (scanned in the block-count scratch)
  uint32_t *gblk = P.blkcnt, *gtot = P.blkcnt + nblk;
  hipLaunchKernelGGL(k_group_mark, dim3(ge), dim3(256), 0, st, P.sc, P.clevel, P.cpbegin,
                     P.cpcount, P.cfchild, P.cnchild, (uint32_t)group_max, group_merge, r,
                     P.pinfo);
  hipLaunchKernelGGL(k_group_count, dim3(nblk), dim3(kB), 0, st, (uint32_t)n, P.pinfo, gblk);
  launch_scan_rows(gblk, nblk, 1, gtot, P.scan, st);
  hipLaunchKernelGGL(k_group_emit, dim3(nblk), dim3(kB), 0, st, (uint32_t)n, P.pinfo, gblk,
                     P.gbegin, P.gid);
  hipLaunchKernelGGL(k_group_total, dim3(1), dim3(64), 0, st, gtot, (uint32_t)n, P.sc,
                     P.gbegin);
  hipLaunchKernelGGL(k_group_size, dim3(ge), dim3(256), 0, st, P.sc, P.gbegin, P.gcount);
  if (r > 0)
    hipLaunchKernelGGL(k_group_root, dim3(ge), dim3(256), 0, st, P.sc, P.gbegin, P.sysoff, nsys,
                       r, P.groot);
}


}  // namespace nb
