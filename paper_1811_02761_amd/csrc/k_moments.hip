// k_moments.hip -- monopole moments of every cell ("calcNode", Sec. 2.2).
//
// M_J and S_J = sum m x are FP64: a leaf sums its particles sequentially in
// key order; an internal cell adds its children's unrounded sums in octant
// order. Stored once rounded: m32 = (float)M, com = (float)(S / M). The size
// b_J of Eq. 2 is read as the largest distance from com to a member
// particle: b2 = max over members of fmaf(dz,dz,fmaf(dy,dy,dx*dx)) with
// d = x - com in FP32; q = (G m32) b2 (FP32) is the left side of Eq. 2 times
// d^4.
//
// Four phases, each over data the previous one finished:
//  1. leaves: one workgroup per block of 256 sorted particles stages them
//     (and a halo) in LDS with coalesced loads; the lane of each leaf's first
//     particle sums the leaf and takes its b2 and q;
//  2. internal cells, deepest level first (their sums need the children's);
//  3. b2 of internal cells: every particle visits all its internal ancestors
//     at once. The level-l ancestor of sorted particle i is found without
//     walking parent links: cells are numbered by level, then by first
//     particle, so its index is the level's offset plus the number of level-l
//     cells starting at or before i (per-level block offsets kept from the
//     build, ballots inside the block) minus one. Lanes sharing an ancestor
//     form runs; each run's maximum is merged by one atomic max on the
//     cell's b2 bit pattern (b2 >= 0: float order = unsigned order; max is
//     order-free, so the result is exact);
//  4. q of internal cells.
// The phases are separated either by kernel boundaries (one launch per
// level in phase 2, the same count of grid-wide synchronisations as the
// paper's calcNode, App. A) or by a lock-free grid barrier inside one
// persistent launch (Xiao and Feng 2010, the method GOTHIC uses).
#include <algorithm>

#include "nbody_internal.h"

namespace nb {

constexpr int kMB = kBuildThreads;          // particles per workgroup (the build's block)
constexpr int kMTile = kMB + kBuildHalo;    // staged particles: block + halo
constexpr int kMWaves = kMB / 64;

// ---------------------------------------------------------------- phase 1
// Sums, com, b2 and q of the leaves starting in block `blk`.
__device__ void leaf_block(uint32_t blk, uint32_t n, float G, DevScalars *__restrict__ sc,
                           const uint32_t *__restrict__ pinfo,
                           const uint32_t *__restrict__ leafof,
                           const uint32_t *__restrict__ cpcount,
                           const float4 *__restrict__ xyzm, double4 *__restrict__ mom64,
                           float4 *__restrict__ nodeA, float4 *__restrict__ nodeB,
                           float4 *tile) {
  const uint32_t b0 = blk * kMB;
  for (int t = threadIdx.x; t < kMTile; t += kMB) {
    const uint32_t p = b0 + (uint32_t)t;
    tile[t] = p < n ? xyzm[p] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  __syncthreads();
  const uint32_t i = b0 + threadIdx.x;
  const uint32_t pi = i < n ? pinfo[i] : 0u;
  const int s = pi & 31, D = (pi >> 5) & 31;
  // i starts its leaf iff it starts a cell at its leaf level D
  if (i < n && s <= D) {
    const uint32_t ncell = sc->ncell;
    const uint32_t leaf = leafof[i];
    const uint32_t cnt = leaf < ncell ? cpcount[leaf] : 0u;
    if (cnt == 0u || cnt > n - i) {
      atomicOr(&sc->status, kStCorrupt);
    } else {
      const uint32_t t0 = threadIdx.x;
      double mm = 0.0, xx = 0.0, yy = 0.0, zz = 0.0;
      for (uint32_t k = 0; k < cnt; ++k) {
        const float4 q = t0 + k < (uint32_t)kMTile ? tile[t0 + k] : xyzm[i + k];
        const double m = (double)q.w;
        mm += m;
        xx += m * (double)q.x;
        yy += m * (double)q.y;
        zz += m * (double)q.z;
      }
      float cx, cy, cz;
      if (mm > 0.0) {
        cx = (float)(xx / mm);
        cy = (float)(yy / mm);
        cz = (float)(zz / mm);
      } else {
        const float4 q = tile[t0];
        cx = q.x;
        cy = q.y;
        cz = q.z;
      }
      float bb = 0.0f;
      for (uint32_t k = 0; k < cnt; ++k) {
        const float4 q = t0 + k < (uint32_t)kMTile ? tile[t0 + k] : xyzm[i + k];
        const float dx = q.x - cx, dy = q.y - cy, dz = q.z - cz;
        const float d2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
        bb = d2 > bb ? d2 : bb;
      }
      const float m32 = (float)mm;
      const float gm = G * m32;
      mom64[leaf] = make_double4(mm, xx, yy, zz);
      nodeA[leaf] = make_float4(cx, cy, cz, bb);
      *reinterpret_cast<float2 *>(&nodeB[leaf]) = make_float2(m32, gm * bb);
    }
  }
}

// ---------------------------------------------------------------- phase 2
// Sums and com of internal cell c from its children; b2 starts at 0.
__device__ __forceinline__ void internal_cell(uint32_t c, uint32_t ncell,
                                              DevScalars *__restrict__ sc,
                                              const uint32_t *__restrict__ cpbegin,
                                              const int32_t *__restrict__ cfchild,
                                              const int32_t *__restrict__ cnchild,
                                              const float4 *__restrict__ xyzm,
                                              double4 *__restrict__ mom64,
                                              float4 *__restrict__ nodeA,
                                              float4 *__restrict__ nodeB) {
  const int k = cnchild[c];
  if (k == 0) return;
  const int32_t f = cfchild[c];
  if (f <= (int32_t)c || k > 8 || (uint32_t)(f + k) > ncell) {
    atomicOr(&sc->status, kStCorrupt);
    return;
  }
  double mm = 0.0, xx = 0.0, yy = 0.0, zz = 0.0;
  for (int q = 0; q < k; ++q) {
    const double4 s = mom64[f + q];
    mm += s.x;
    xx += s.y;
    yy += s.z;
    zz += s.w;
  }
  float cx, cy, cz;
  if (mm > 0.0) {
    cx = (float)(xx / mm);
    cy = (float)(yy / mm);
    cz = (float)(zz / mm);
  } else {
    const float4 p = xyzm[cpbegin[c]];
    cx = p.x;
    cy = p.y;
    cz = p.z;
  }
  mom64[c] = make_double4(mm, xx, yy, zz);
  nodeA[c] = make_float4(cx, cy, cz, 0.0f);
  nodeB[c].x = (float)mm;
}

// ---------------------------------------------------------------- phase 3
struct B2Shared {
  uint64_t wbal[kMWaves][kLevels];  // per wave and level: lanes starting a level-l cell
  uint32_t wpre[kLevels][kMWaves];  // per level: starts in the block's earlier waves
  uint32_t lvl_off[kLevels + 1];
};

// Wave64 maximum of unsigned values by DPP (all lanes active): max within
// rows of 16 by row_shr 1, 2, 4, 8 (zero fill: values are >= 0), then rows
// 1 and 3 take row 0 and 2's last lane (row_bcast:15), rows 2 and 3 lane 31
// (row_bcast:31); lane 63 then holds the maximum.
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

__device__ __forceinline__ void b2_merge(float4 *__restrict__ nodeA, uint32_t c, uint32_t v) {
  uint32_t *w = reinterpret_cast<uint32_t *>(&nodeA[c].w);
  if (v > *w) atomicMax(w, v);
}

// b2 contributions of the particles of block `blk` to their internal
// ancestors. Wave-uniform control flow throughout (DPP and ballots).
__device__ void b2_block(uint32_t blk, uint32_t n, uint32_t nblk, uint32_t ncell,
                         DevScalars *__restrict__ sc, const uint32_t *__restrict__ pinfo,
                         const uint32_t *__restrict__ lvlblk, const float4 *__restrict__ xyzm,
                         float4 *__restrict__ nodeA, B2Shared &S) {
  const uint32_t i = blk * kMB + threadIdx.x;
  const bool valid = i < n;
  const uint32_t pi = valid ? pinfo[i] : 0u;
  const int s = pi & 31, D = (pi >> 5) & 31;
  const int w = threadIdx.x >> 6;
  const uint32_t lane = lane_id();
  for (int l = 0; l < kLevels; ++l) {
    const uint64_t b = __ballot(valid && s <= l && l <= D);
    if (lane == 0) S.wbal[w][l] = b;
  }
  if (threadIdx.x <= kLevels) S.lvl_off[threadIdx.x] = sc->lvl_off[threadIdx.x];
  __syncthreads();
  if (threadIdx.x < kLevels) {
    uint32_t o = 0;
    for (int q = 0; q < kMWaves; ++q) {
      S.wpre[threadIdx.x][q] = o;
      o += (uint32_t)__popcll(S.wbal[q][threadIdx.x]);
    }
  }
  __syncthreads();
  const float4 p = valid ? xyzm[i] : make_float4(0.f, 0.f, 0.f, 0.f);
  const uint64_t le = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  const int top = (int)__builtin_amdgcn_readfirstlane(wave_max_u32(valid ? (uint32_t)D : 0u));
  for (int l = 0; l < top; ++l) {
    const bool act = valid && l < D;  // the level-l ancestor is internal
    const uint64_t am = __ballot(act);
    if (am == 0) continue;
    const uint64_t sm = S.wbal[w][l];
    const uint32_t base = S.lvl_off[l] + lvlblk[(size_t)l * nblk + blk] + S.wpre[l][w];
    const uint32_t anc = base + (uint32_t)__popcll(sm & le) - 1u;
    uint32_t v = 0u;
    if (act) {
      if (anc < ncell) {
        const float4 c = nodeA[anc];
        const float dx = p.x - c.x, dy = p.y - c.y, dz = p.z - c.z;
        v = __float_as_uint(__builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx)));
      } else {
        atomicOr(&sc->status, kStCorrupt);
      }
    }
    // runs of lanes sharing an ancestor begin at an active lane that starts
    // a level-l cell, or at lane 0 (an active lane after an inactive one
    // always starts a cell: the particle before it is in no level-l
    // internal cell)
    uint64_t heads = am & (sm | 1ull);
    const int nh = __popcll(heads);
    if (nh <= 3) {
      while (heads) {
        const int h = __builtin_ctzll(heads);
        heads &= heads - 1;
        const uint64_t upto = heads ? (heads & (~heads + 1ull)) - 1ull : ~0ull;  // lanes < next head
        const uint64_t run = am & upto & (~0ull << h);
        const bool in = (run >> lane) & 1ull;
        const uint32_t mx = wave_max_dpp(in ? v : 0u);
        if (lane == (uint32_t)h && anc < ncell) b2_merge(nodeA, anc, mx);
      }
    } else {
      // segmented inclusive maximum: start lane of each run, then the max
      const bool head = (heads >> lane) & 1ull;
      uint32_t st = head ? lane : 0u;
      for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(st, d, 64);
        if (lane >= (uint32_t)d && o > st) st = o;
      }
      for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(v, d, 64);
        if (lane >= st + (uint32_t)d && o > v) v = o;
      }
      const bool nxt_head = lane < 63 && ((heads >> (lane + 1)) & 1ull);
      const bool nxt_act = lane < 63 && ((am >> (lane + 1)) & 1ull);
      if (act && (lane == 63 || nxt_head || !nxt_act) && anc < ncell) b2_merge(nodeA, anc, v);
    }
  }
}

// ---------------------------------------------------------------- phase 4
__device__ __forceinline__ void internal_q(uint32_t c, float G, const float4 *__restrict__ nodeA,
                                           float4 *__restrict__ nodeB) {
  const float4 b = nodeB[c];
  if (__float_as_uint(b.w) & kLeafBit) return;  // leaves are finished by phase 1
  const float gm = G * b.x;
  nodeB[c].y = gm * nodeA[c].w;
}

// ------------------------------------------------ one launch per phase/level
__global__ __launch_bounds__(kMB) void k_mom_leaf(DevScalars *__restrict__ sc, uint32_t n,
                                                  float G, const uint32_t *__restrict__ pinfo,
                                                  const uint32_t *__restrict__ leafof,
                                                  const uint32_t *__restrict__ cpcount,
                                                  const float4 *__restrict__ xyzm,
                                                  double4 *__restrict__ mom64,
                                                  float4 *__restrict__ nodeA,
                                                  float4 *__restrict__ nodeB) {
  __shared__ float4 tile[kMTile];
  leaf_block(blockIdx.x, n, G, sc, pinfo, leafof, cpcount, xyzm, mom64, nodeA, nodeB, tile);
}

__global__ __launch_bounds__(256) void k_mom_level(DevScalars *__restrict__ sc, int level,
                                                   const uint32_t *__restrict__ cpbegin,
                                                   const int32_t *__restrict__ cfchild,
                                                   const int32_t *__restrict__ cnchild,
                                                   const float4 *__restrict__ xyzm,
                                                   double4 *__restrict__ mom64,
                                                   float4 *__restrict__ nodeA,
                                                   float4 *__restrict__ nodeB) {
  const uint32_t ncell = sc->ncell;
  if (ncell == 0) return;
  const uint32_t c0 = sc->lvl_off[level], c1 = sc->lvl_off[level + 1];
  for (uint32_t c = c0 + blockIdx.x * blockDim.x + threadIdx.x; c < c1;
       c += gridDim.x * blockDim.x)
    internal_cell(c, ncell, sc, cpbegin, cfchild, cnchild, xyzm, mom64, nodeA, nodeB);
}

__global__ __launch_bounds__(kMB) void k_mom_b2(DevScalars *__restrict__ sc, uint32_t n,
                                                uint32_t nblk,
                                                const uint32_t *__restrict__ pinfo,
                                                const uint32_t *__restrict__ lvlblk,
                                                const float4 *__restrict__ xyzm,
                                                float4 *__restrict__ nodeA) {
  __shared__ B2Shared S;
  b2_block(blockIdx.x, n, nblk, sc->ncell, sc, pinfo, lvlblk, xyzm, nodeA, S);
}

__global__ __launch_bounds__(256) void k_mom_q(const DevScalars *__restrict__ sc, float G,
                                               const float4 *__restrict__ nodeA,
                                               float4 *__restrict__ nodeB) {
  const uint32_t nc = sc->ncell;
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x)
    internal_q(c, G, nodeA, nodeB);
}

// ------------------------------------------------- one persistent launch
// Lock-free grid barrier (Xiao and Feng 2010): each workgroup publishes its
// arrival in in[wg]; workgroup 0 waits for every arrival and then releases
// each workgroup through out[wg]. Goals grow monotonically (an epoch per
// launch, bumped on the device by the kernel before, times 64, plus the
// barrier's number), so the flags are never reset; each launch of
// k_mom_grid passes at most 63 barriers. Waits are bounded: a workgroup
// that spins past kSpinLimit latches kStCorrupt and all its lanes leave the
// kernel (the others then time out too), so the launch always ends.
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

__global__ __launch_bounds__(kMB) void k_mom_grid(
    DevScalars *__restrict__ sc, uint32_t n, uint32_t nblk, float G,
    const uint32_t *__restrict__ pinfo, const uint32_t *__restrict__ leafof,
    const uint32_t *__restrict__ lvlblk, const uint32_t *__restrict__ cpbegin,
    const uint32_t *__restrict__ cpcount, const int32_t *__restrict__ cfchild,
    const int32_t *__restrict__ cnchild, const float4 *__restrict__ xyzm,
    double4 *__restrict__ mom64, float4 *__restrict__ nodeA, float4 *__restrict__ nodeB,
    unsigned long long *bar_in, unsigned long long *bar_out) {
  __shared__ union {
    float4 tile[kMTile];
    B2Shared b2;
  } sm;
  __shared__ int fail;
  if (threadIdx.x == 0) fail = 0;
  __syncthreads();
  unsigned long long goal = sc->bar_epoch * 64ull;
  const uint32_t ncell = sc->ncell;
  for (uint32_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    leaf_block(b, n, G, sc, pinfo, leafof, cpcount, xyzm, mom64, nodeA, nodeB, sm.tile);
    __syncthreads();
  }
  if (!grid_sync(bar_in, bar_out, ++goal, &fail, sc)) return;
  // the deepest level holding cells has leaves only
  int top = 0;
  for (int l = 0; l < kLevels; ++l)
    if (sc->lvl_off[l + 1] > sc->lvl_off[l]) top = l;
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x, nth = gridDim.x * blockDim.x;
  for (int l = top - 1; l >= 0; --l) {
    const uint32_t c0 = sc->lvl_off[l], c1 = sc->lvl_off[l + 1];
    for (uint32_t c = c0 + tid; c < c1; c += nth)
      internal_cell(c, ncell, sc, cpbegin, cfchild, cnchild, xyzm, mom64, nodeA, nodeB);
    if (!grid_sync(bar_in, bar_out, ++goal, &fail, sc)) return;
  }
  for (uint32_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    b2_block(b, n, nblk, ncell, sc, pinfo, lvlblk, xyzm, nodeA, sm.b2);
    __syncthreads();
  }
  if (!grid_sync(bar_in, bar_out, ++goal, &fail, sc)) return;
  for (uint32_t c = tid; c < ncell; c += nth) internal_q(c, G, nodeA, nodeB);
}

void launch_moments(int64_t n, float G, const Ptrs &P, const Layout &L, int mode,
                    hipStream_t st) {
  const uint32_t nblk = (uint32_t)cdiv(n, kMB);
  if (mode == kCalcNodeGrid) {
    const uint32_t g = (uint32_t)std::min<int64_t>(std::max<int64_t>(L.num_cu, 1), kBarSlots);
    hipLaunchKernelGGL(k_bar_epoch, dim3(1), dim3(1), 0, st, P.sc);
    hipLaunchKernelGGL(k_mom_grid, dim3(g), dim3(kMB), 0, st, P.sc, (uint32_t)n, nblk, G,
                       P.pinfo, P.leafof, P.lvlblk, P.cpbegin, P.cpcount, P.cfchild,
                       P.cnchild, P.xyzm, P.mom64, P.nodeA, P.nodeB, P.bar, P.bar + kBarSlots);
    return;
  }
  hipLaunchKernelGGL(k_mom_leaf, dim3(nblk), dim3(kMB), 0, st, P.sc, (uint32_t)n, G, P.pinfo,
                     P.leafof, P.cpcount, P.xyzm, P.mom64, P.nodeA, P.nodeB);
  int64_t gl = cdiv(n, 256 * 4);
  if (gl > 2048) gl = 2048;
  if (gl < 1) gl = 1;
  for (int l = kMaxLevel - 1; l >= 0; --l)
    hipLaunchKernelGGL(k_mom_level, dim3(gl), dim3(256), 0, st, P.sc, l, P.cpbegin,
                       P.cfchild, P.cnchild, P.xyzm, P.mom64, P.nodeA, P.nodeB);
  hipLaunchKernelGGL(k_mom_b2, dim3(nblk), dim3(kMB), 0, st, P.sc, (uint32_t)n, nblk, P.pinfo,
                     P.lvlblk, P.xyzm, P.nodeA);
  int64_t gc = cdiv(L.cell_cap, 256);
  if (gc > 4096) gc = 4096;
  if (gc < 1) gc = 1;
  hipLaunchKernelGGL(k_mom_q, dim3(gc), dim3(256), 0, st, P.sc, G, P.nodeA, P.nodeB);
}

}  // namespace nb
