// k_sort.hip -- stable LSD radix sort of (63-bit key, 32-bit index) pairs.
//
// The paper's tree build spends most of its time in a key/value radix sort
// (Sec. 4.1). This is a reduce-then-scan LSD sort with 8-bit digits and 8
// passes, written for wave64: every pass is a per-tile digit histogram (LDS
// atomics), a per-digit exclusive scan over tiles, and a scatter whose
// in-tile rank comes from a wave-level multisplit (eight ballots give the
// lanes sharing a digit; their popcount below the lane is the rank). Ranks
// follow input position, so each pass is stable and equal keys keep their
// input order.
#include "nbody_internal.h"

namespace nb {

constexpr int kWaves = kSortThreads / 64;
// the scatter of a 4096-key tile runs 8 wavefronts of 8 keys per lane: two
// tiles (58 KB of LDS each) per CU keep 16 wavefronts resident (4 with 16
// keys per lane waited on the rank chain; 59 vs 73 us per pass at 2^23)
constexpr int kScatterThreads = 512;
constexpr int kWaveKeys = kSortTile / kWaves;  // 1024 keys per wave

// Lanes whose digit equals this lane's digit (among `valid` lanes).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint64_t valid) {
  uint64_t peers = valid;
#pragma unroll
  for (int b = 0; b < kSortBits; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

// Per-tile digit counts by LDS atomics (one per key, into the wave's own
// counters; the order of the additions does not matter).
__global__ __launch_bounds__(kSortThreads) void k_sort_hist(
    const uint64_t *__restrict__ keys, int64_t n, int shift, uint32_t *__restrict__ hist,
    int64_t nblk, const uint32_t *__restrict__ n_dev) {
  if (n_dev) n = min(n, (int64_t)*n_dev);  // a count known on the device only
  __shared__ uint32_t cnt[kWaves][kSortRadix];
  for (int t = threadIdx.x; t < kWaves * kSortRadix; t += kSortThreads) (&cnt[0][0])[t] = 0;
  __syncthreads();
  const int w = threadIdx.x >> 6;
  const int64_t base = blockIdx.x * (int64_t)kSortTile + w * kWaveKeys + lane_id();
#pragma unroll
  for (int it = 0; it < kWaveKeys / 64; ++it) {
    const int64_t i = base + it * 64;
    if (i < n) atomicAdd(&cnt[w][(uint32_t)(keys[i] >> shift) & (kSortRadix - 1)], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < kSortRadix; d += kSortThreads) {
    uint32_t s = 0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) s += cnt[q][d];
    hist[d * nblk + blockIdx.x] = s;
  }
}

// Block-wide exclusive scan of one value per thread (blockDim = kSortThreads).
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *tot,
                                                    uint32_t *wsum) {
  const uint32_t inc = wave_incl_scan(v);
  const int w = threadIdx.x >> 6;
  if (lane_id() == 63) wsum[w] = inc;
  __syncthreads();
  uint32_t off = 0, all = 0;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
    if (q < w) off += wsum[q];
    all += wsum[q];
  }
  if (tot) *tot = all;
  __syncthreads();
  return off + inc - v;
}

// One workgroup per digit: exclusive scan of hist[d][0..nblk) in place and
// the digit total.
__global__ __launch_bounds__(kSortThreads) void k_sort_scan(uint32_t *__restrict__ hist,
                                                             int64_t nblk,
                                                             uint32_t *__restrict__ totals) {
  __shared__ uint32_t wsum[kWaves];
  uint32_t *row = hist + blockIdx.x * nblk;
  const int64_t per = cdiv(nblk, kSortThreads);
  const int64_t b0 = threadIdx.x * per;
  uint32_t s = 0;
  for (int64_t k = b0; k < b0 + per && k < nblk; ++k) s += row[k];
  uint32_t tot;
  uint32_t run = block_excl_scan(s, &tot, wsum);
  for (int64_t k = b0; k < b0 + per && k < nblk; ++k) {
    const uint32_t v = row[k];
    row[k] = run;
    run += v;
  }
  if (threadIdx.x == 0) totals[blockIdx.x] = tot;
}

// Scatter of one tile: ranks as in the histogram pass (stable: wave, item,
// lane = input order), then the tile is reordered by digit in LDS and
// written out from there, so consecutive threads store consecutive
// addresses of each digit's run instead of 256 scattered runs per wave.
template <int kThreads>
__global__ __launch_bounds__(kThreads) void k_sort_scatter(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin, int64_t n,
    int shift, const uint32_t *__restrict__ hist, int64_t nblk,
    const uint32_t *__restrict__ totals, uint64_t *__restrict__ kout,
    uint32_t *__restrict__ vout, const uint32_t *__restrict__ n_dev) {
  constexpr int kW = kThreads / 64;
  constexpr int kItems = kSortTile / kThreads;
  constexpr int kWK = kSortTile / kW;
  static_assert(kThreads >= kSortRadix, "one thread per digit");
  if (n_dev) n = min(n, (int64_t)*n_dev);
  __shared__ uint32_t cnt[kW][kSortRadix];
  __shared__ uint32_t dbase[kSortRadix];   // global start of each digit's run of this tile
  __shared__ uint32_t lstart[kSortRadix];  // tile-local start of each digit
  __shared__ uint32_t wsum[kW];
  __shared__ uint64_t sk[kSortTile];
  __shared__ uint32_t sv[kSortTile];
  for (int t = threadIdx.x; t < kW * kSortRadix; t += kThreads) (&cnt[0][0])[t] = 0;
  // digit start = exclusive scan of totals; plus this tile's offset
  {
    const bool dig = threadIdx.x < (unsigned)kSortRadix;
    const uint32_t tv = dig ? totals[threadIdx.x] : 0u;
    const uint32_t ex = block_excl_scan(tv, nullptr, wsum);
    if (dig) dbase[threadIdx.x] = ex + hist[threadIdx.x * nblk + blockIdx.x];
  }
  __syncthreads();
  const int w = threadIdx.x >> 6;
  const int64_t tile0 = blockIdx.x * (int64_t)kSortTile;
  const int64_t base = tile0 + w * kWK;
  uint64_t k[kItems];
  uint32_t v[kItems];
  uint32_t r[kItems];
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const int64_t i = base + it * 64 + lane_id();
    const bool valid = i < n;
    const uint64_t vmask = __ballot(valid);
    k[it] = valid ? kin[i] : 0ull;
    v[it] = valid ? vin[i] : 0u;
    const uint32_t d = (uint32_t)(k[it] >> shift) & (kSortRadix - 1);
    const uint64_t peers = match_digit(d, vmask);
    const uint32_t below = (uint32_t)__popcll(peers & lanemask_lt());
    uint32_t c0 = 0;
    if (valid) c0 = cnt[w][d];
    r[it] = c0 + below;
    // every lane has read the counter before the digit's first lane bumps it
    __builtin_amdgcn_wave_barrier();
    if (valid && below == 0) cnt[w][d] = c0 + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  // per digit: offsets of the waves within the tile's digit, then the
  // digit's start within the tile
  uint32_t tot = 0;
  if (threadIdx.x < (unsigned)kSortRadix) {
    const int d = threadIdx.x;
    uint32_t o = 0;
#pragma unroll
    for (int q = 0; q < kW; ++q) {
      const uint32_t t = cnt[q][d];
      cnt[q][d] = o;
      o += t;
    }
    tot = o;
  }
  const uint32_t ls = block_excl_scan(tot, nullptr, wsum);
  if (threadIdx.x < (unsigned)kSortRadix) lstart[threadIdx.x] = ls;
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const int64_t i = base + it * 64 + lane_id();
    if (i < n) {
      const uint32_t d = (uint32_t)(k[it] >> shift) & (kSortRadix - 1);
      const uint32_t lp = lstart[d] + cnt[w][d] + r[it];
      sk[lp] = k[it];
      sv[lp] = v[it];
    }
  }
  __syncthreads();
  const int64_t m = min((int64_t)kSortTile, n - tile0);  // valid items of the tile
  for (int j = threadIdx.x; j < m; j += kThreads) {
    const uint64_t key = sk[j];
    const uint32_t d = (uint32_t)(key >> shift) & (kSortRadix - 1);
    const uint32_t pos = dbase[d] + ((uint32_t)j - lstart[d]);
    kout[pos] = key;
    vout[pos] = sv[j];
  }
}

void launch_digit_sort(int64_t n, const uint32_t *n_dev, int shift, const uint64_t *kin,
                       const uint32_t *vin, uint64_t *kout, uint32_t *vout, uint32_t *hist,
                       hipStream_t st) {
  const int64_t nblk = cdiv(n, kSortTile);
  uint32_t *totals = hist + (int64_t)kSortRadix * nblk;
  hipLaunchKernelGGL(k_sort_hist, dim3(nblk), dim3(kSortThreads), 0, st, kin, n, shift, hist,
                     nblk, n_dev);
  hipLaunchKernelGGL(k_sort_scan, dim3(kSortRadix), dim3(kSortThreads), 0, st, hist, nblk,
                     totals);
  hipLaunchKernelGGL(k_sort_scatter<kScatterThreads>, dim3(nblk), dim3(kScatterThreads), 0, st,
                     kin, vin, n, shift, hist, nblk, totals, kout, vout, n_dev);
}

void launch_sort(int64_t n, uint64_t *keysA, uint32_t *valsA, uint64_t *keysB,
                 uint32_t *valsB, uint32_t *hist, hipStream_t st, uint64_t **keys_out,
                 uint32_t **vals_out) {
  const int64_t nblk = cdiv(n, kSortTile);
  uint32_t *totals = hist + (int64_t)kSortRadix * nblk;
  uint64_t *ki = keysA, *ko = keysB;
  uint32_t *vi = valsA, *vo = valsB;
  for (int pass = 0; pass < 8; ++pass) {
    launch_digit_sort(n, nullptr, pass * kSortBits, ki, vi, ko, vo, hist, st);
    uint64_t *tk = ki; ki = ko; ko = tk;
    uint32_t *tv = vi; vi = vo; vo = tv;
  }
  *keys_out = ki;
  *vals_out = vi;
}

}  // namespace nb
