// k_moments.hip -- monopole moments of every cell ("calcNode", Sec. 2.2).
//
// M_J and S_J = sum m x are FP64: a leaf sums its particles sequentially in
// key order (starting from 0); an internal cell adds its children's
// unrounded sums in octant order. Stored once rounded: m32 = (float)M,
// com = (float)(S / M). The size b_J of Eq. 2 is read as the largest
// distance from com to a member particle: b2 = max over members of
// fmaf(dz,dz,fmaf(dy,dy,dx*dx)) with d = x - com in FP32; q = (G m32) b2
// (FP32) is the left side of Eq. 2 times d^4.
//
// Phases, each over data the previous ones finished:
//  1. leaves: one lane per leaf (the build lists the leaves in particle
//     order; a wavefront's 64 leaves are contiguous, so their particles are
//     staged in LDS with coalesced loads): sums, com, b2, q.
//  2. internal sums, deepest level first, over the build's per-level lists of
//     internal cells (the children's sums must be final). Planned from the
//     per-level counts of the latest tree the host has seen: a level with
//     more than kNarrowCells internal cells gets a launch of its own (the
//     grid-wide synchronisation of the paper's calcNode, App. A); a run of
//     consecutive levels with fewer runs in one workgroup, with workgroup
//     barriers between its levels. Without counts: one launch per level. Or
//     (a selectable variant) one persistent launch with a lock-free grid
//     barrier between levels (Xiao and Feng 2010, the method GOTHIC uses).
//  3. b2 of internal cells. A cell of at most 64 particles: a half
//     wavefront, two particles per lane at most. A bigger cell: a pass over
//     the sorted particles, every
//     particle meeting each of its big cells. The level-l cell of sorted
//     particle i is found without parent links: cells are numbered by level,
//     then by first particle, so its index is the level's offset plus the
//     number of level-l cells starting at or before i, minus one (counts
//     before a wavefront's range are kept from the build per block of 256
//     particles; inside it they are ballots). A big cell spans more than 64
//     particles, so 64 consecutive particles meet at most one start of a big
//     cell per level: at most two runs of lanes per level, each reduced by a
//     DPP maximum; a run reaching lane 63 is carried into the next 64
//     particles, and each finished run is merged by an atomic max on the
//     cell's b2 bit pattern (b2 >= 0: float order = unsigned order; max is
//     order-free, so the result is exact).
//  4. q of internal cells.
#include <algorithm>

#include "nbody_internal.h"

namespace nb {

constexpr int kChunksPerWave = 16;
constexpr uint32_t kWaveSpan = 64u * kChunksPerWave;  // sorted particles per wavefront
static_assert(kWaveSpan % kBuildThreads == 0, "wavefront ranges start at build blocks");
constexpr uint32_t kNoCell = 0xffffffffu;
constexpr uint32_t kSmallCell = 64;   // bigger cells go to the particle pass (the build's E)
constexpr uint32_t kLeafStage = 512;  // particles staged per wavefront in the leaf pass

// Lanes 0 .. lane (inclusive) as a mask.
__device__ __forceinline__ uint64_t lanes_le(uint32_t lane) {
  return lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
}

// Wave64 maximum of unsigned values by DPP (all lanes active): rows of 16 by
// row_shr 1, 2, 4, 8 (zero fill: values are >= 0), then row_bcast:15 and
// row_bcast:31; lane 63 holds the maximum.
__device__ __forceinline__ uint32_t wave_max_dpp(uint32_t v) {
  int x = (int)v;
  x = max((uint32_t)x, (uint32_t)__builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true));
  x = max((uint32_t)x, (uint32_t)__builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true));
  x = max((uint32_t)x, (uint32_t)__builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true));
  x = max((uint32_t)x, (uint32_t)__builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true));
  x = max((uint32_t)x, (uint32_t)__builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false));
  x = max((uint32_t)x, (uint32_t)__builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false));
  return (uint32_t)__builtin_amdgcn_readlane(x, 63);
}

__device__ __forceinline__ float dist2(float4 p, float cx, float cy, float cz) {
  const float dx = p.x - cx, dy = p.y - cy, dz = p.z - cz;
  return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
}

// com of sums (M, S): S / M rounded once; a cell without mass takes its
// first particle's position.
__device__ __forceinline__ float3 com_of(double M, double Sx, double Sy, double Sz,
                                         float4 first) {
  if (M > 0.0) return make_float3((float)(Sx / M), (float)(Sy / M), (float)(Sz / M));
  return make_float3(first.x, first.y, first.z);
}

// ---------------------------------------------------------------- phase 1
__global__ __launch_bounds__(256) void k_mom_leaf(DevScalars *__restrict__ sc, uint32_t n,
                                                  float G, const uint2 *__restrict__ leaves,
                                                  const float4 *__restrict__ xyzm,
                                                  double4 *__restrict__ mom64,
                                                  float4 *__restrict__ nodeA,
                                                  float4 *__restrict__ nodeB) {
  __shared__ float4 stage[4][kLeafStage];
  const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
  const uint32_t nleaf = sc->nleaf, ncell = sc->ncell;
  const uint32_t k0 = (blockIdx.x * 4u + w) * 64u;
  if (k0 >= nleaf) return;  // wave-uniform
  const uint32_t k = k0 + lane;
  const bool has = k < nleaf;
  const uint2 e = has ? leaves[k] : make_uint2(0u, 0u);
  // a leaf ends where the next one begins (the leaves tile the particles)
  const uint32_t pb = e.y;
  const uint32_t pe = has ? (k + 1u < nleaf ? leaves[k + 1u].y : n) : 0u;
  const uint32_t kl = min(nleaf - 1u, k0 + 63u) - k0;  // last lane with a leaf
  const uint32_t P0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)pb);
  const uint32_t P1 = (uint32_t)__builtin_amdgcn_readlane((int)pe, (int)kl);
  const uint32_t span = (P1 > P0 && P1 <= n) ? min(P1 - P0, kLeafStage) : 0u;
  {  // all loads in flight before the LDS stores (a rolled loop waited on each)
    float4 tmp[kLeafStage / 64];
#pragma unroll
    for (uint32_t u = 0; u < kLeafStage / 64; ++u) {
      const uint32_t t = lane + 64u * u;
      tmp[u] = t < span ? xyzm[P0 + t] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (uint32_t u = 0; u < kLeafStage / 64; ++u) {
      const uint32_t t = lane + 64u * u;
      if (t < span) stage[w][t] = tmp[u];
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (!has) return;
  if (e.x >= ncell || pe <= pb || pe > n || pb < P0) {
    atomicOr(&sc->status, kStCorrupt);
    return;
  }
  double mm = 0.0, xx = 0.0, yy = 0.0, zz = 0.0;
#pragma unroll 4
  for (uint32_t p = pb; p < pe; ++p) {
    const float4 q = p - P0 < span ? stage[w][p - P0] : xyzm[p];
    const double m = (double)q.w;  // m x is exact in FP64 (two 24-bit significands)
    mm += m;
    xx += m * (double)q.x;
    yy += m * (double)q.y;
    zz += m * (double)q.z;
  }
  const float3 c = com_of(mm, xx, yy, zz, pb - P0 < span ? stage[w][pb - P0] : xyzm[pb]);
  float bb = 0.0f;
#pragma unroll 4
  for (uint32_t p = pb; p < pe; ++p) {
    const float d2 = dist2(p - P0 < span ? stage[w][p - P0] : xyzm[p], c.x, c.y, c.z);
    bb = d2 > bb ? d2 : bb;
  }
  const float m32 = (float)mm;
  const float gm = G * m32;
  mom64[e.x] = make_double4(mm, xx, yy, zz);
  nodeA[e.x] = make_float4(c.x, c.y, c.z, bb);
  *reinterpret_cast<float2 *>(&nodeB[e.x]) = make_float2(m32, gm * bb);
}

// ---------------------------------------------------------------- phase 2
// Internal cell e = (cell, first child, children, particles): its sums from
// the children's, in octant order; com and m32; b2 starts at 0.
__device__ __forceinline__ void internal_cell(uint4 e, uint32_t ncell, uint32_t n,
                                              DevScalars *sc,
                                              const uint32_t *__restrict__ cpbegin,
                                              const float4 *__restrict__ xyzm,
                                              double4 *__restrict__ mom64,
                                              float4 *__restrict__ nodeA,
                                              float4 *__restrict__ nodeB) {
  const uint32_t c = e.x, f = e.y, k = e.z;
  if (c >= ncell || k == 0u || k > 8u || f <= c || f + k > ncell) {
    atomicOr(&sc->status, kStCorrupt);
    return;
  }
  double4 ch[8];
#pragma unroll
  for (uint32_t q = 0; q < 8; ++q)
    if (q < k) ch[q] = mom64[f + q];
  double mm = 0.0, xx = 0.0, yy = 0.0, zz = 0.0;
#pragma unroll
  for (uint32_t q = 0; q < 8; ++q) {
    if (q < k) {
      mm += ch[q].x;
      xx += ch[q].y;
      yy += ch[q].z;
      zz += ch[q].w;
    }
  }
  float4 first = make_float4(0.f, 0.f, 0.f, 0.f);
  if (!(mm > 0.0)) {
    const uint32_t pb = cpbegin[c];
    if (pb < n) first = xyzm[pb];
    else atomicOr(&sc->status, kStCorrupt);
  }
  const float3 cm = com_of(mm, xx, yy, zz, first);
  mom64[c] = make_double4(mm, xx, yy, zz);
  nodeA[c] = make_float4(cm.x, cm.y, cm.z, 0.0f);
  nodeB[c].x = (float)mm;
}

__global__ __launch_bounds__(256) void k_mom_level(DevScalars *__restrict__ sc, int level,
                                                   uint32_t n, const uint4 *__restrict__ ilist,
                                                   const uint32_t *__restrict__ cpbegin,
                                                   const float4 *__restrict__ xyzm,
                                                   double4 *__restrict__ mom64,
                                                   float4 *__restrict__ nodeA,
                                                   float4 *__restrict__ nodeB) {
  const uint32_t ncell = sc->ncell;
  const uint32_t t0 = sc->istart[level], t1 = sc->istart[level + 1];
  for (uint32_t t = t0 + blockIdx.x * blockDim.x + threadIdx.x; t < t1;
       t += gridDim.x * blockDim.x)
    internal_cell(ilist[t], ncell, n, sc, cpbegin, xyzm, mom64, nodeA, nodeB);
}

// Several consecutive levels with few internal cells (lo <= l <= hi,
// deepest first) in one workgroup: a workgroup barrier between levels.
__global__ __launch_bounds__(1024) void k_mom_levels_narrow(DevScalars *__restrict__ sc, int lo,
                                                            int hi, uint32_t n,
                                                            const uint4 *__restrict__ ilist,
                                                            const uint32_t *__restrict__ cpbegin,
                                                            const float4 *__restrict__ xyzm,
                                                            double4 *__restrict__ mom64,
                                                            float4 *__restrict__ nodeA,
                                                            float4 *__restrict__ nodeB) {
  const uint32_t ncell = sc->ncell;
  for (int l = hi; l >= lo; --l) {
    const uint32_t t0 = sc->istart[l], t1 = sc->istart[l + 1];
    for (uint32_t t = t0 + threadIdx.x; t < t1; t += blockDim.x)
      internal_cell(ilist[t], ncell, n, sc, cpbegin, xyzm, mom64, nodeA, nodeB);
    __syncthreads();  // (makes the level's global writes visible to the workgroup)
  }
}

// Lock-free grid barrier (Xiao and Feng 2010): each workgroup publishes its
// arrival in in[wg]; workgroup 0 waits for every arrival and then releases
// each workgroup through out[wg]. Goals grow monotonically (an epoch per
// launch, bumped on the device by the kernel before, times 64, plus the
// barrier's number), so the flags are never reset; a launch passes at most
// 22 barriers. Waits are bounded: a workgroup that spins past kSpinLimit
// latches kStCorrupt and leaves the kernel (the others then time out too),
// so the launch always ends.
constexpr uint32_t kSpinLimit = 1u << 22;

__device__ bool grid_sync(unsigned long long *bar_in, unsigned long long *bar_out,
                          unsigned long long goal, int *fail, DevScalars *sc) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();  // this workgroup's writes before its arrival
    __hip_atomic_store(&bar_in[blockIdx.x], goal, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (blockIdx.x == 0) {
    for (uint32_t t = threadIdx.x; t < gridDim.x; t += blockDim.x) {
      uint32_t k = 0;
      while (__hip_atomic_load(&bar_in[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < goal) {
        if (++k > kSpinLimit) {
          *fail = 1;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __syncthreads();
    if (!*fail) {
      __threadfence();
      for (uint32_t t = threadIdx.x; t < gridDim.x; t += blockDim.x)
        __hip_atomic_store(&bar_out[t], goal, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (threadIdx.x == 0 && !*fail) {
    uint32_t k = 0;
    while (__hip_atomic_load(&bar_out[blockIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
           goal) {
      if (++k > kSpinLimit) {
        *fail = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __threadfence();  // the other workgroups' writes after the release
  }
  __syncthreads();
  if (*fail) {
    if (threadIdx.x == 0) atomicOr(&sc->status, kStCorrupt);
    return false;
  }
  return true;
}

__global__ void k_bar_epoch(DevScalars *sc) { sc->bar_epoch += 1ull; }

// Phase 2 in one persistent launch: every level, deepest first, then a grid
// barrier. The grid holds no more workgroups than can be resident at once.
__global__ __launch_bounds__(256) void k_mom_levels_grid(DevScalars *__restrict__ sc, uint32_t n,
                                                         const uint4 *__restrict__ ilist,
                                                         const uint32_t *__restrict__ cpbegin,
                                                         const float4 *__restrict__ xyzm,
                                                         double4 *__restrict__ mom64,
                                                         float4 *__restrict__ nodeA,
                                                         float4 *__restrict__ nodeB,
                                                         unsigned long long *bar_in,
                                                         unsigned long long *bar_out) {
  __shared__ int fail;
  if (threadIdx.x == 0) fail = 0;
  __syncthreads();
  unsigned long long goal = sc->bar_epoch * 64ull;
  const uint32_t ncell = sc->ncell;
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x, nth = gridDim.x * blockDim.x;
  for (int l = kMaxLevel - 1; l >= 0; --l) {
    const uint32_t t0 = sc->istart[l], t1 = sc->istart[l + 1];
    if (t1 <= t0) continue;  // uniform over the grid: no barrier needed
    for (uint32_t t = t0 + tid; t < t1; t += nth)
      internal_cell(ilist[t], ncell, n, sc, cpbegin, xyzm, mom64, nodeA, nodeB);
    if (!grid_sync(bar_in, bar_out, ++goal, &fail, sc)) return;
  }
}

// ---------------------------------------------------------------- phase 3
// b2 of the internal cells of at most kSmallCell particles: 32 lanes per
// cell (two particles per lane at most), coalesced loads, then a maximum
// over the half wavefront.
__global__ __launch_bounds__(256) void k_mom_b2small(DevScalars *__restrict__ sc, uint32_t n,
                                                     const uint4 *__restrict__ ilist,
                                                     const uint32_t *__restrict__ cpbegin,
                                                     const float4 *__restrict__ xyzm,
                                                     float4 *__restrict__ nodeA) {
  const uint32_t ncell = sc->ncell, total = sc->istart[kLevels];
  const uint32_t lane = lane_id(), h = lane & 31u;
  const uint32_t nhalf = gridDim.x * (blockDim.x >> 5);
  for (uint32_t t0 = (blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 2u; t0 < total;
       t0 += nhalf) {
    const uint32_t t = t0 + (lane >> 5);  // this half's cell
    uint4 e = make_uint4(0u, 0u, 0u, 0u);
    if (t < total) e = ilist[t];
    const bool mine = t < total && e.w <= kSmallCell;
    uint32_t pb = 0u;
    float4 cm = make_float4(0.f, 0.f, 0.f, 0.f);
    if (mine) {
      pb = e.x < ncell ? cpbegin[e.x] : n;
      if (pb >= n || e.w == 0u || e.w > n - pb) {
        if (h == 0) atomicOr(&sc->status, kStCorrupt);
        pb = n;
      } else {
        cm = nodeA[e.x];
      }
    }
    const bool ok = mine && pb < n;
    uint32_t v = 0u;
    if (ok && h < e.w) v = __float_as_uint(dist2(xyzm[pb + h], cm.x, cm.y, cm.z));
    if (ok && h + 32u < e.w) {
      const uint32_t v2 = __float_as_uint(dist2(xyzm[pb + h + 32u], cm.x, cm.y, cm.z));
      v = v2 > v ? v2 : v;
    }
    // maximum over each half (b2 >= 0: the bit patterns order like the values)
    for (int d = 1; d < 32; d <<= 1) {
      const uint32_t o = (uint32_t)__shfl_xor((int)v, d, 64);
      v = o > v ? o : v;
    }
    if (ok && h == 0) reinterpret_cast<float *>(&nodeA[e.x])[3] = __uint_as_float(v);
  }
}

__device__ __forceinline__ void b2_merge(float4 *__restrict__ nodeA, uint32_t c, uint32_t v) {
  uint32_t *w = reinterpret_cast<uint32_t *>(&nodeA[c].w);
  if (v > *w) atomicMax(w, v);
}

// b2 of the internal cells of more than kSmallCell particles: particle i
// meets its cells at levels 0 .. T_i = min(E_i, D_i - 1). Lane l of a
// wavefront keeps level l's state: the level's offset plus the count of
// level-l cells starting before the next particle (so the index of the cell
// starting next) and the carried run (cell, maximum). At the start of every
// 64 particles lane l also fetches the centre of mass of the level-l cell
// they continue (one load for all levels).
__global__ __launch_bounds__(256) void k_mom_b2big(DevScalars *__restrict__ sc, uint32_t n,
                                                   uint32_t nblk,
                                                   const uint32_t *__restrict__ pinfo,
                                                   const uint32_t *__restrict__ lvlblk,
                                                   const float4 *__restrict__ xyzm,
                                                   float4 *__restrict__ nodeA) {
  const uint32_t lane = lane_id();
  const uint32_t wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const uint64_t r0 = (uint64_t)wave * kWaveSpan;
  if (r0 >= n) return;  // wave-uniform
  const uint32_t r1 = (uint32_t)std::min<uint64_t>(n, r0 + kWaveSpan);
  const uint32_t ncell = sc->ncell;
  const uint64_t le = lanes_le(lane);
  uint32_t base = 0;
  if (lane < (uint32_t)kLevels)
    base = sc->lvl_off[lane] + lvlblk[(size_t)lane * nblk + r0 / kBuildThreads];
  uint32_t ccell = kNoCell, cmax = 0u;
  uint32_t npi = 0u;
  float4 np = make_float4(0.f, 0.f, 0.f, 0.f);
  {
    const uint32_t i = (uint32_t)r0 + lane;
    if (i < r1) {
      npi = pinfo[i];
      np = xyzm[i];
    }
  }
  for (uint32_t c0 = (uint32_t)r0; c0 < r1; c0 += 64u) {
    const uint32_t i = c0 + lane;
    const bool valid = i < r1;
    const uint32_t pi = npi;
    const float4 p = np;
    if (c0 + 64u < r1) {  // the next 64 particles, while these are processed
      const uint32_t j = i + 64u;
      npi = j < r1 ? pinfo[j] : 0u;
      np = j < r1 ? xyzm[j] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    const int s = pi & 31, D = (pi >> 5) & 31, E = (int)((pi >> 10) & 31u) - 1;
    const int T = valid ? min(E, D - 1) : -1;
    const uint32_t starts = (valid && s <= D) ? ((2u << D) - (1u << s)) : 0u;  // bit l: starts a level-l cell
    const int top = (int)wave_max_dpp((uint32_t)(T + 1)) - 1;
    const int dtop = (int)wave_max_dpp(valid ? (uint32_t)D + 1u : 0u) - 1;
    // carried runs of levels no big cell here reaches have ended
    if (lane < (uint32_t)kLevels && (int)lane > top && ccell != kNoCell) {
      b2_merge(nodeA, ccell, cmax);
      ccell = kNoCell;
    }
    // lane l <= top: centre of mass of the level-l cell continued from before
    float4 cc = make_float4(0.f, 0.f, 0.f, 0.f);
    if ((int)lane <= top && base - 1u < ncell) cc = nodeA[base - 1u];
    for (int l = 0; l <= dtop; ++l) {
      const uint64_t Sa = __ballot((starts >> l) & 1u);  // level-l cell starts
      const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)base, l);
      if (lane == (uint32_t)l) base = b + (uint32_t)__popcll(Sa);
      if (l > top) continue;
      const bool act = l <= T;
      const uint64_t A = __ballot(act);
      const uint64_t S = Sa & A;  // starts of big level-l cells
      const uint32_t ccl = (uint32_t)__builtin_amdgcn_readlane((int)ccell, l);
      const uint32_t cml = (uint32_t)__builtin_amdgcn_readlane((int)cmax, l);
      uint32_t nc = kNoCell, nm = 0u;
      if (S == 0ull) {
        // one run: the lanes continuing cell b - 1 (some lane reaches l)
        const uint32_t cell = b - 1u;
        const float cx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cc.x), l));
        const float cy = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cc.y), l));
        const float cz = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cc.z), l));
        uint32_t mx = wave_max_dpp(act ? __float_as_uint(dist2(p, cx, cy, cz)) : 0u);
        if (ccl == cell) {
          mx = max(mx, cml);
        } else if (ccl != kNoCell && lane == 0) {
          b2_merge(nodeA, ccl, cml);
        }
        if (cell >= ncell) {
          if (lane == 0) atomicOr(&sc->status, kStCorrupt);
        } else if ((A >> 63) & 1ull) {
          nc = cell;
          nm = mx;
        } else if (lane == 0) {
          b2_merge(nodeA, cell, mx);
        }
      } else {
        // a big cell starts here (a big cell spans more than 64 particles:
        // at most one start, but any number is handled): runs from lane 0
        // (continuing cell b - 1, if lane 0 is active) and from each start
        const bool cont = (A & 1ull) && !(S & 1ull);
        if (ccl != kNoCell && (!cont || ccl != b - 1u) && lane == 0) b2_merge(nodeA, ccl, cml);
        const uint32_t keep = (cont && ccl == b - 1u) ? cml : 0u;
        uint64_t st = S;
        int h = cont ? -1 : __builtin_ctzll(st);
        if (!cont) st &= st - 1ull;
        for (;;) {
          const uint64_t upto = st ? ((st & (~st + 1ull)) - 1ull) : ~0ull;
          const uint64_t from = h < 0 ? ~0ull : (~0ull << h);
          const uint64_t msk = A & upto & from;
          const uint32_t cell =
              h < 0 ? b - 1u : b + (uint32_t)__popcll(Sa & lanes_le((uint32_t)h)) - 1u;
          if (cell < ncell) {
            const float4 cmv = nodeA[cell];
            const bool in = (msk >> lane) & 1ull;
            uint32_t mx =
                wave_max_dpp(in ? __float_as_uint(dist2(p, cmv.x, cmv.y, cmv.z)) : 0u);
            if (h < 0) mx = max(mx, keep);
            if ((msk >> 63) & 1ull) {
              nc = cell;
              nm = mx;
            } else if (lane == 0) {
              b2_merge(nodeA, cell, mx);
            }
          } else if (lane == 0) {
            atomicOr(&sc->status, kStCorrupt);
          }
          if (!st) break;
          h = __builtin_ctzll(st);
          st &= st - 1ull;
        }
      }
      if (lane == (uint32_t)l) {
        ccell = nc;
        cmax = nm;
      }
    }
    // levels past every particle's leaf here: their carried runs ended too
    if (lane < (uint32_t)kLevels && (int)lane > dtop && ccell != kNoCell) {
      b2_merge(nodeA, ccell, cmax);
      ccell = kNoCell;
    }
  }
  // runs open at the end of the range may go on past it
  if (lane < (uint32_t)kLevels && ccell != kNoCell) b2_merge(nodeA, ccell, cmax);
}

// ---------------------------------------------------------------- phase 4
__global__ __launch_bounds__(256) void k_mom_q(const DevScalars *__restrict__ sc, float G,
                                               const uint4 *__restrict__ ilist,
                                               const float4 *__restrict__ nodeA,
                                               float4 *__restrict__ nodeB) {
  const uint32_t ncell = sc->ncell, total = sc->istart[kLevels];
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += gridDim.x * blockDim.x) {
    const uint32_t c = ilist[t].x;
    if (c >= ncell) continue;
    const float gm = G * nodeB[c].x;
    nodeB[c].y = gm * nodeA[c].w;
  }
}

namespace {
// Workgroups of the persistent phase-2 launch: one per compute unit (all
// resident at once, as the barrier needs; fewer arrivals for workgroup 0 to
// poll than a fully occupied grid), at most kBarSlots.
int grid_blocks(int num_cu) { return std::min(std::max(num_cu, 1), kBarSlots); }
}  // namespace

void launch_moments(int64_t n, float G, const Ptrs &P, const Layout &L, int mode,
                    const uint32_t *level_cells, hipStream_t st) {
  const uint32_t nblk = (uint32_t)cdiv(n, kBuildThreads);
  // leaves <= n: one wavefront per 64 leaves, four per workgroup
  hipLaunchKernelGGL(k_mom_leaf, dim3((uint32_t)cdiv(n, 256)), dim3(256), 0, st, P.sc,
                     (uint32_t)n, G, P.leaves, P.xyzm, P.mom64, P.nodeA, P.nodeB);
  if (mode == kCalcNodeGrid) {
    hipLaunchKernelGGL(k_bar_epoch, dim3(1), dim3(1), 0, st, P.sc);
    hipLaunchKernelGGL(k_mom_levels_grid, dim3(grid_blocks(L.num_cu)), dim3(256), 0, st, P.sc,
                       (uint32_t)n, P.ilist, P.cpbegin, P.xyzm, P.mom64, P.nodeA, P.nodeB,
                       P.bar, P.bar + kBarSlots);
  } else {
    int64_t gl = cdiv(n, 256 * 8);
    gl = std::min<int64_t>(std::max<int64_t>(gl, 1), 2048);
    // with level_cells (internal cells per level of a recent tree) runs of
    // levels with at most kNarrowCells cells go to one single-workgroup
    // launch each (correct for any counts; only the speed depends on them)
    int hi = -1;  // top of the open run of narrow levels
    for (int l = kMaxLevel - 1; l >= 0; --l) {
      const bool narrow = level_cells && level_cells[l] <= kNarrowCells;
      if (narrow) {
        if (hi < 0) hi = l;
        if (l > 0) continue;
      }
      if (hi >= 0) {
        const int lo = narrow ? l : l + 1;
        hipLaunchKernelGGL(k_mom_levels_narrow, dim3(1), dim3(1024), 0, st, P.sc, lo, hi,
                           (uint32_t)n, P.ilist, P.cpbegin, P.xyzm, P.mom64, P.nodeA,
                           P.nodeB);
        hi = -1;
      }
      if (!narrow)
        hipLaunchKernelGGL(k_mom_level, dim3(gl), dim3(256), 0, st, P.sc, l, (uint32_t)n,
                           P.ilist, P.cpbegin, P.xyzm, P.mom64, P.nodeA, P.nodeB);
    }
  }
  int64_t gi = cdiv(n, 256 * 4);
  gi = std::min<int64_t>(std::max<int64_t>(gi, 1), 4096);
  hipLaunchKernelGGL(k_mom_b2small, dim3(gi), dim3(256), 0, st, P.sc, (uint32_t)n, P.ilist,
                     P.cpbegin, P.xyzm, P.nodeA);
  const uint32_t waves = (uint32_t)cdiv(n, kWaveSpan);
  hipLaunchKernelGGL(k_mom_b2big, dim3((uint32_t)cdiv(waves, 4)), dim3(256), 0, st, P.sc,
                     (uint32_t)n, nblk, P.pinfo, P.lvlblk, P.xyzm, P.nodeA);
  hipLaunchKernelGGL(k_mom_q, dim3(gi), dim3(256), 0, st, P.sc, G, P.ilist, P.nodeA, P.nodeB);
}

}  // namespace nb
