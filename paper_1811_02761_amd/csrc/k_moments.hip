// k_moments.hip -- monopole moments of every cell ("calcNode", Sec. 2.2).
//
// M_J and S_J = sum m x are FP64: a leaf sums its particles sequentially in
// key order; an internal cell adds its children's unrounded sums in octant
// order. Stored once rounded: m32 = (float)M, com = (float)(S / M). The size
// b_J of Eq. 2 is read as the largest distance from com to a member
// particle: b2 = max over members of fmaf(dz,dz,fmaf(dy,dy,dx*dx)) with
// d = x - com in FP32; q = (G m32) b2 (FP32) is the left side of Eq. 2 times
// d^4. Levels are processed deepest first, one launch per level (the paper's
// calcNode likewise synchronises the whole grid once per level, App. A).
#include "nbody_internal.h"

namespace nb {

__device__ __forceinline__ float4 com_from(double M, double Sx, double Sy, double Sz,
                                           float4 first) {
  if (M > 0.0) return make_float4((float)(Sx / M), (float)(Sy / M), (float)(Sz / M), 0.f);
  return make_float4(first.x, first.y, first.z, 0.f);
}

__global__ __launch_bounds__(256) void k_mom_leaf(DevScalars *__restrict__ sc, uint32_t n,
                                                  const uint32_t *__restrict__ cpbegin,
                                                  const uint32_t *__restrict__ cpcount,
                                                  const int32_t *__restrict__ cnchild,
                                                  const float4 *__restrict__ xyzm,
                                                  double4 *__restrict__ mom64,
                                                  float4 *__restrict__ nodeA,
                                                  float4 *__restrict__ nodeB) {
  const uint32_t nc = sc->ncell;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nc;
       c += (int64_t)gridDim.x * blockDim.x) {
    if (cnchild[c] != 0) continue;
    const uint32_t b = cpbegin[c], e = b + cpcount[c];
    if (b >= n || e > n || e <= b) {
      atomicOr(&sc->status, kStCorrupt);
      continue;
    }
    // four particles per trip: their loads are issued together; the sums
    // still run over the particles one by one in key order
    constexpr uint32_t U = 4;
    double mm = 0.0, xx = 0.0, yy = 0.0, zz = 0.0;
    for (uint32_t i0 = b; i0 < e; i0 += U) {
      float4 q[U];
#pragma unroll
      for (uint32_t u = 0; u < U; ++u) q[u] = xyzm[i0 + u < e ? i0 + u : b];
#pragma unroll
      for (uint32_t u = 0; u < U; ++u) {
        if (i0 + u >= e) break;
        const double m = (double)q[u].w;
        mm += m;
        xx += m * (double)q[u].x;
        yy += m * (double)q[u].y;
        zz += m * (double)q[u].z;
      }
    }
    const float4 com = com_from(mm, xx, yy, zz, xyzm[b]);
    float bb = 0.0f;
    for (uint32_t i0 = b; i0 < e; i0 += U) {
      float4 q[U];
#pragma unroll
      for (uint32_t u = 0; u < U; ++u) q[u] = xyzm[i0 + u < e ? i0 + u : b];
#pragma unroll
      for (uint32_t u = 0; u < U; ++u) {
        if (i0 + u >= e) break;
        const float dx = q[u].x - com.x, dy = q[u].y - com.y, dz = q[u].z - com.z;
        const float d2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
        bb = d2 > bb ? d2 : bb;
      }
    }
    mom64[c] = make_double4(mm, xx, yy, zz);
    nodeA[c] = make_float4(com.x, com.y, com.z, bb);
    nodeB[c].x = (float)mm;
  }
}

__global__ __launch_bounds__(256) void k_mom_level(DevScalars *__restrict__ sc,
                                                   int level,
                                                   const uint32_t *__restrict__ cpbegin,
                                                   const int32_t *__restrict__ cfchild,
                                                   const int32_t *__restrict__ cnchild,
                                                   const float4 *__restrict__ xyzm,
                                                   double4 *__restrict__ mom64,
                                                   float4 *__restrict__ nodeA,
                                                   float4 *__restrict__ nodeB) {
  if (sc->ncell == 0) return;
  const uint32_t c0 = sc->lvl_off[level], c1 = sc->lvl_off[level + 1];
  for (int64_t c = c0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < c1;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int k = cnchild[c];
    if (k == 0) continue;
    const int32_t f = cfchild[c];
    if (f <= (int32_t)c || k > 8 || (uint32_t)(f + k) > sc->ncell) {
      atomicOr(&sc->status, kStCorrupt);
      continue;
    }
    double mm = 0.0, xx = 0.0, yy = 0.0, zz = 0.0;
    for (int q = 0; q < k; ++q) {
      const double4 s = mom64[f + q];
      mm += s.x;
      xx += s.y;
      yy += s.z;
      zz += s.w;
    }
    const float4 com = com_from(mm, xx, yy, zz, xyzm[cpbegin[c]]);
    mom64[c] = make_double4(mm, xx, yy, zz);
    nodeA[c] = make_float4(com.x, com.y, com.z, 0.0f);  // b2 set by k_mom_b2
    nodeB[c].x = (float)mm;
  }
}

// b2 of internal cells: every particle visits its ancestors (leaf excluded),
// deepest first. One wavefront takes kB2Chunks x 64 consecutive particles,
// 64 at a time. At each level the lanes whose ancestor sits at that level
// form runs of equal cell (cells are contiguous particle ranges and numbered
// in particle order); a segmented max over the runs leaves each run's
// maximum in its last lane. A run that reaches lane 63 may go on in the next
// 64 particles: it is carried (lane l of the wave keeps the cell and maximum
// of level l) instead of stored. Every finished run makes one atomic max on
// the cell's bit pattern (b2 >= 0, so the float order equals the unsigned
// order), skipped when the stored value is already as large.
constexpr int kB2Chunks = 16;
constexpr uint32_t kNoCell = 0xffffffffu;

__device__ __forceinline__ void b2_store(float4 *__restrict__ nodeA, uint32_t c, uint32_t v) {
  uint32_t *w = reinterpret_cast<uint32_t *>(&nodeA[c].w);
  if (v > *w) atomicMax(w, v);
}

__global__ __launch_bounds__(256) void k_mom_b2(DevScalars *__restrict__ sc, uint32_t n,
                                                const uint32_t *__restrict__ pinfo,
                                                const uint32_t *__restrict__ leafof,
                                                const int32_t *__restrict__ cparent,
                                                const float4 *__restrict__ xyzm,
                                                float4 *__restrict__ nodeA) {
  const uint32_t lane = lane_id();
  const uint32_t ncell = sc->ncell;
  const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const uint64_t r0 = wave * 64u * kB2Chunks;
  // carried run of level `lane` (lanes 0 .. kMaxLevel - 1)
  uint32_t cc = kNoCell, cm = 0u;
  for (int ch = 0; ch < kB2Chunks; ++ch) {
    const uint64_t i = r0 + (uint64_t)ch * 64u + lane;
    if (r0 + (uint64_t)ch * 64u >= n) break;  // wave-uniform
    const bool valid = i < n;
    float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
    int lvl = -1;
    uint32_t cur = kNoCell;
    if (valid) {
      p = xyzm[i];
      const int D = (pinfo[i] >> 5) & 31;
      const uint32_t lf = leafof[i];
      if (D > 0 && lf < ncell) {
        const int32_t pc = cparent[lf];
        if (pc >= 0 && (uint32_t)pc < ncell) {
          cur = (uint32_t)pc;
          lvl = D - 1;
        } else {
          atomicOr(&sc->status, kStCorrupt);
        }
      }
    }
    const int top = (int)wave_max_u32((uint32_t)(lvl + 1)) - 1;
    // carried runs above this chunk's deepest ancestor level have ended
    if ((int)lane > top && lane < (uint32_t)kMaxLevel && cc != kNoCell) {
      b2_store(nodeA, cc, cm);
      cc = kNoCell;
      cm = 0u;
    }
    for (int l = top; l >= 0; --l) {
      const bool act = lvl == l;
      // inactive lanes get keys of their own (above any cell index)
      const uint32_t key = act ? cur : (kNoCell ^ lane);
      uint32_t v = 0u, up = kNoCell;
      if (act) {
        // the parent index is read with the centre of mass, so that both
        // loads of a level share one memory round trip
        const float4 c = nodeA[cur];
        if (l > 0) up = (uint32_t)cparent[cur];
        const float dx = p.x - c.x, dy = p.y - c.y, dz = p.z - c.z;
        v = __float_as_uint(__builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx)));
      }
      const uint32_t ccl = __builtin_amdgcn_readlane(cc, l);
      const uint32_t cml = __builtin_amdgcn_readlane(cm, l);
      const uint32_t k0 = __builtin_amdgcn_readfirstlane(key);
      const uint32_t k63 = __builtin_amdgcn_readlane(key, 63);
      if (__ballot(act) == ~0ull && k0 == k63) {
        // the whole chunk is one run (the common case above the leaves)
        v = wave_max_u32(v);
        if (ccl == k0) {
          v = cml > v ? cml : v;
        } else if (ccl != kNoCell && lane == 0) {
          b2_store(nodeA, ccl, cml);
        }
        if (lane == (uint32_t)l) {
          cc = k0;
          cm = v;
        }
      } else {
        const uint32_t kprev = __shfl_up(key, 1, 64);
        const uint32_t knext = __shfl_down(key, 1, 64);
        const bool first = lane == 0 || kprev != key;
        const bool last = lane == 63 || knext != key;
        // start lane of each run, then the segmented inclusive max
        uint32_t st = first ? lane : 0u;
        for (int d = 1; d < 64; d <<= 1) {
          const uint32_t o = __shfl_up(st, d, 64);
          if (lane >= (uint32_t)d && o > st) st = o;
        }
        for (int d = 1; d < 64; d <<= 1) {
          const uint32_t o = __shfl_up(v, d, 64);
          if (lane >= st + (uint32_t)d && o > v) v = o;
        }
        // the carried run of level l goes on iff lane 0 continues its cell
        const bool merge = ccl != kNoCell && k0 == ccl;
        if (ccl != kNoCell && !merge && lane == 0) b2_store(nodeA, ccl, cml);
        if (merge && st == 0u && cml > v) v = cml;
        // runs ending before lane 63 are finished; the run at lane 63 is carried
        if (act && last && lane != 63) b2_store(nodeA, key, v);
        const uint32_t v63 = __builtin_amdgcn_readlane(v, 63);
        const bool act63 = k63 < ncell;
        if (lane == (uint32_t)l) {
          cc = act63 ? k63 : kNoCell;
          cm = act63 ? v63 : 0u;
        }
      }
      if (act) {
        if (l > 0 && up >= ncell) {
          atomicOr(&sc->status, kStCorrupt);
          lvl = -1;
        } else {
          cur = up;
          lvl = l - 1;
        }
      }
    }
  }
  if (lane < (uint32_t)kMaxLevel && cc != kNoCell) b2_store(nodeA, cc, cm);
}

__global__ __launch_bounds__(256) void k_mom_final(const DevScalars *__restrict__ sc,
                                                   float G,
                                                   const float4 *__restrict__ nodeA,
                                                   float4 *__restrict__ nodeB) {
  const uint32_t nc = sc->ncell;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nc;
       c += (int64_t)gridDim.x * blockDim.x) {
    const float gm = G * nodeB[c].x;
    nodeB[c].y = gm * nodeA[c].w;
  }
}

void launch_moments(int64_t n, float G, const Ptrs &P, const Layout &L, hipStream_t st) {
  int64_t gc = cdiv(L.cell_cap, 256);
  if (gc > 4096) gc = 4096;
  if (gc < 1) gc = 1;
  hipLaunchKernelGGL(k_mom_leaf, dim3(gc), dim3(256), 0, st, P.sc, (uint32_t)n, P.cpbegin, P.cpcount,
                     P.cnchild, P.xyzm, P.mom64, P.nodeA, P.nodeB);
  int64_t gl = cdiv(n, 256 * 4);
  if (gl > 2048) gl = 2048;
  if (gl < 1) gl = 1;
  for (int l = kMaxLevel - 1; l >= 0; --l)
    hipLaunchKernelGGL(k_mom_level, dim3(gl), dim3(256), 0, st, P.sc, l, P.cpbegin,
                       P.cfchild, P.cnchild, P.xyzm, P.mom64, P.nodeA, P.nodeB);
  hipLaunchKernelGGL(k_mom_b2, dim3(cdiv(n, 4 * 64 * kB2Chunks)), dim3(256), 0, st, P.sc,
                     (uint32_t)n, P.pinfo, P.leafof, P.cparent, P.xyzm, P.nodeA);
  hipLaunchKernelGGL(k_mom_final, dim3(gc), dim3(256), 0, st, P.sc, G, P.nodeA, P.nodeB);
}

}  // namespace nb
